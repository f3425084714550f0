// Transform kernels: pruned z-column passes, xy-plane passes with fused
// pointwise work, and full-grid passes (gfx950).
#include "fft_lds.h"
#include "kernels.h"

namespace lgw {

namespace {

constexpr int kZCols = 32;           // z-columns per workgroup in column passes

#ifndef LGW_PLANE_THREADS_48
#define LGW_PLANE_THREADS_48 256
#endif
template <int N> constexpr int plane_threads() { return N >= 64 ? 512 : (N == 48 ? LGW_PLANE_THREADS_48 : 256); }

// every kernel here runs at least 256 threads, more than the longest table
template <typename T, int N>
__device__ __forceinline__ void load_tw(cplx<T>* tw_s, const cplx<T>* tw) {
  static_assert(N <= 256, "one table entry per thread");
  if (threadIdx.x < N) tw_s[threadIdx.x] = tw[threadIdx.x];
}

// The same in two halves, so that a kernel can issue the load ahead of its
// other loads and store it once it is needed (a load and its LDS store in one
// place make every later load wait for it).  Threads past the table load
// entry 0 and drop it.
template <typename T, int N>
__device__ __forceinline__ cplx<T> get_tw(const cplx<T>* tw) {
  static_assert(N <= 256, "one table entry per thread");
  return tw[threadIdx.x < N ? threadIdx.x : 0];
}
template <typename T, int N>
__device__ __forceinline__ void put_tw(cplx<T>* tw_s, cplx<T> v) {
  if (threadIdx.x < N) tw_s[threadIdx.x] = v;
}

// sequence t of a pruned set {-h..h} mapped to its index mod N
template <int N>
__device__ __forceinline__ int pruned(int t, int h) { return t <= h ? t : t + N - 2 * h - 1; }

// buf[cl * LDZ + skew(z)] = src[z * ld + c0 + cl] for z < N, cl < nc, in two
// halves: all of a thread's loads (zcols_load), later its LDS stores
// (zcols_store); a loop that stores each value before the next load waits on
// memory once per element.
template <int N> constexpr int zcols_per_thread() { return (N * kZCols + 255) / 256; }
template <typename T, int N>
__device__ __forceinline__ void zcols_load(const cplx<T>* __restrict__ src, long ld, int c0, int nc,
                                           cplx<T> (&v)[zcols_per_thread<N>()]) {
#pragma unroll
  for (int k = 0; k < zcols_per_thread<N>(); ++k) {
    const int i = threadIdx.x + k * 256;
    const int ii = i < N * nc ? i : 0;   // element (0, 0) exists; its copy is not stored
    const int z = ii / nc, cl = ii - z * nc;
    v[k] = src[(long)z * ld + c0 + cl];
  }
}
template <typename T, int N>
__device__ __forceinline__ void zcols_store(cplx<T>* buf, int nc, const cplx<T> (&v)[zcols_per_thread<N>()]) {
  constexpr int LDZ = skew(N) + 1;
#pragma unroll
  for (int k = 0; k < zcols_per_thread<N>(); ++k) {
    const int i = threadIdx.x + k * 256;
    if (i < N * nc) {
      const int z = i / nc, cl = i - z * nc;
      buf[cl * LDZ + skew(z)] = v[k];
    }
  }
}

// ------------------------------------------------------------------ zinv
// With partial projector sums (f.part != null) X is the direction D, and the
// projected input f.pre .* D - sum_v Phi_v C_v is formed in the gather and
// also stored to Xout.
// FED selects the variant at compile time, so that the plain pass keeps its
// registers.
template <typename T, int N, bool FED>
__global__ void __launch_bounds__(256)
k_zinv(Geom g, const cplx<T>* __restrict__ tw, const cplx<T>* X, long ldx,
       cplx<T>* __restrict__ Tb, long ldt, T scale, const int* __restrict__ act, ProjFeed<T> f,
       cplx<T>* __restrict__ Xout) {
  constexpr int LDZ = skew(N) + 1;
  // points of the block's run per thread whose loads are issued ahead
  constexpr int KZ = sizeof(T) == 4 ? 4 : 2;
  // partial sums per lane loaded ahead (at most 64 slices over 8 lanes)
  constexpr int KP = 8;
  __shared__ cplx<T> buf[kZCols * LDZ];
  __shared__ cplx<T> tws[N];
  __shared__ cplx<T> Cs[kMaxBands];
  const int sys = sys_of(act, blockIdx.y);
  const int c0 = blockIdx.x * kZCols;
  const int nc = min(kZCols, g.ncols - c0);
  const cplx<T>* Xs = X + (long)sys * ldx;
  cplx<T>* Ts = Tb + (long)sys * ldt;
  __shared__ int cs[kZCols + 1];
  __shared__ int ch[kZCols];
  // the block's columns are one contiguous run [run0, run1) of the sphere vector
  const int run0 = g.col_start[c0];
  const int run1 = c0 + nc < g.ncols ? g.col_start[c0 + nc] : g.npw;
  // Everything a thread reads from global memory that does not depend on
  // another load is issued first, in the order it is needed (the memory
  // latency is paid about once rather than once per dependent step): the
  // twiddles and column table, the partial sums and the scalars of the
  // direction update, the fed transform's point data.  Out-of-range slots
  // load a valid element (entry 0, column c0, run0, slice 0) and drop it.
  const cplx<T> twv = get_tw<T, N>(tw);
  const int cq = threadIdx.x < nc ? threadIdx.x : 0;
  const int csv = g.col_start[c0 + cq], chv = g.col_h[c0 + cq];
  T th = T(-1), rrv = T(1);
  cplx<T> cpv{0, 0};
  cplx<T> pp[KP];
  cplx<T> pf_ph[KZ][8], pf_r[KZ], pf_d[KZ];
  T pf_sc[KZ];
  [[maybe_unused]] const int v = threadIdx.x >> 3, l = threadIdx.x & 7;
  if constexpr (FED) {
    static_assert(kMaxBands * 8 == 256, "eight lanes per band over the workgroup");
    if (f.r) {
      th = f.theta[sys];
      rrv = f.rr[sys];
      if (l == 0 && v < f.nv) cpv = f.Cp[(long)sys * f.nv + v];
    }
#pragma unroll
    for (int q = 0; q < KP; ++q) {
      const int k = l + 8 * q;
      const bool ok = v < f.nv && k < f.nsplit;
      pp[q] = f.part[ok ? ((long)k * f.ntot + sys) * f.nv + v : 0];
    }
#pragma unroll
    for (int k = 0; k < KZ; ++k) {
      const int gi = run0 + threadIdx.x + k * 256;
      const int gs = gi < run1 ? gi : run0;
      pf_sc[k] = f.pre ? f.pre[gs] : T(1);
#pragma unroll
      for (int u = 0; u < 8; ++u) pf_ph[k][u] = u < f.nv ? f.Phi[(long)u * f.ldphi + gs] : cplx<T>{0, 0};
      pf_d[k] = Xs[gs];
      pf_r[k] = f.r ? f.r[(long)sys * ldx + gs] : cplx<T>{0, 0};
    }
  }
  put_tw<T, N>(tws, twv);
  if (threadIdx.x < nc) {
    cs[threadIdx.x] = csv;
    ch[threadIdx.x] = chv;
  }
  if (threadIdx.x == 0) cs[nc] = run1;
  for (int i = threadIdx.x; i < kZCols * LDZ; i += 256) buf[i] = cplx<T>{0, 0};
  if constexpr (FED) {
    // this system's projector coefficients, the sum of its slices: eight
    // lanes per band (kMaxBands * 8 = 256 threads), then a shuffle tree
    cplx<T> a{0, 0};
    if (v < f.nv) {
#pragma unroll
      for (int q = 0; q < KP; ++q)
        if (l + 8 * q < f.nsplit) a = a + pp[q];
      for (int k = l + 8 * KP; k < f.nsplit; k += 8) a = a + f.part[((long)k * f.ntot + sys) * f.nv + v];
    }
#pragma unroll
    for (int o = 4; o > 0; o >>= 1) {
      a.x += __shfl_xor(a.x, o, 64);
      a.y += __shfl_xor(a.y, o, 64);
    }
    if (l == 0 && v < f.nv) {
      // with the direction update, part holds the residual's sums:
      // C(p) = C(r) + beta C(p_old)
      if (f.r && th >= T(0)) a = a + (th / rrv) * cpv;
      Cs[v] = a;
      if (f.r && blockIdx.x == 0) f.Cn[(long)sys * f.nv + v] = a;
    }
  }
  // direction update: p = r + beta p while a new norm is parked in theta
  // (with r set, the direction X is p itself)
  bool upd = false;
  T beta = T(0);
  if constexpr (FED) {
    upd = f.r && th >= T(0);
    if (upd) beta = th / rrv;
  }
  __syncthreads();
  // one point of the run: the column it belongs to, its value, its slot in
  // the column buffer
  auto put = [&](int gi, cplx<T> xv) {
    int lo = 0, hi = nc;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (cs[mid] <= gi) lo = mid; else hi = mid;
    }
    const int mz = gi - cs[lo] - ch[lo];
    buf[lo * LDZ + skew(mz < 0 ? mz + N : mz)] = xv;
  };
  if constexpr (FED) {
    auto fed_point = [&](int gi, const cplx<T> (&ph)[8], T sc, cplx<T> rv, cplx<T> dv) {
      cplx<T> xv;
      if (upd) {
        xv = rv + beta * dv;
        f.p[(long)sys * ldx + gi] = xv;
      } else {
        xv = dv;
      }
      xv = sc * xv;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (u < f.nv) xv = xv - Cs[u] * ph[u];
      for (int w = 8; w < f.nv; ++w) xv = xv - Cs[w] * f.Phi[(long)w * f.ldphi + gi];
      Xout[(long)sys * ldx + gi] = xv;
      put(gi, xv);
    };
#pragma unroll
    for (int k = 0; k < KZ; ++k) {
      const int gi = run0 + threadIdx.x + k * 256;
      if (gi < run1) fed_point(gi, pf_ph[k], pf_sc[k], pf_r[k], pf_d[k]);
    }
    for (int gi = run0 + threadIdx.x + KZ * 256; gi < run1; gi += 256) {
      cplx<T> ph[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) ph[u] = u < f.nv ? f.Phi[(long)u * f.ldphi + gi] : cplx<T>{0, 0};
      const T sc = f.pre ? f.pre[gi] : T(1);
      const cplx<T> rv = f.r ? f.r[(long)sys * ldx + gi] : cplx<T>{0, 0};
      fed_point(gi, ph, sc, rv, Xs[gi]);
    }
  } else {
    for (int gi = run0 + threadIdx.x; gi < run1; gi += 256) put(gi, Xs[gi]);
  }
  __syncthreads();
  fft_lds<T, N, +1, 256, kZCols, false>(buf, tws, nc, [](int t, int e) { return t * LDZ + skew(e); });
  for (int i = threadIdx.x; i < N * nc; i += 256) {
    const int z = i / nc, cl = i - z * nc;
    Ts[(long)z * g.ncols + c0 + cl] = scale * buf[cl * LDZ + skew(z)];
  }
}

// ------------------------------------------------------------------ zfwd
// sum over the 256 threads of a column workgroup (the total in every thread)
template <typename T>
__device__ __forceinline__ T zblock_sum(T v, T* sm) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  return (sm[0] + sm[1]) + (sm[2] + sm[3]);
}

// MODE 0: plain; 1: CG step work (CgDot); 2: projector coefficients of the
// stored Y per column workgroup (ProjPart, at most 8 bands).
template <typename T, int N, int MODE>
__global__ void __launch_bounds__(256)
k_zfwd(Geom g, const cplx<T>* __restrict__ tw, const cplx<T>* __restrict__ Tb, long ldt, T scale,
       const cplx<T>* __restrict__ X, long ldx, const cplx<T>* __restrict__ shift,
       const cplx<T>* __restrict__ E, long lde, const T* __restrict__ ecoef,
       cplx<T>* __restrict__ Y, long ldy, const int* __restrict__ act, const T* __restrict__ dout,
       CgDot<T> cd, ProjPart<T> pp) {
  constexpr bool DOT = MODE == 1;
  constexpr bool PDOT = MODE == 2;
  constexpr int LDZ = skew(N) + 1;
  // points of the block's run per thread whose operands are loaded before
  // the transform (not with PDOT, whose band rows would take the registers)
  constexpr int KZ = PDOT ? 0 : (sizeof(T) == 4 ? 4 : 2);
  __shared__ cplx<T> buf[kZCols * LDZ];
  __shared__ cplx<T> tws[N];
  const int sys = sys_of(act, blockIdx.y);
  const int c0 = blockIdx.x * kZCols;
  const int nc = min(kZCols, g.ncols - c0);
  const cplx<T>* Ts = Tb + (long)sys * ldt;
  __shared__ int cs[kZCols + 1];
  __shared__ int ch[kZCols];
  const int run0 = g.col_start[c0];
  const int run1 = c0 + nc < g.ncols ? g.col_start[c0 + nc] : g.npw;
  // loads issued in the order they are needed (see k_zinv)
  const cplx<T> twv = get_tw<T, N>(tw);
  const int cq = threadIdx.x < nc ? threadIdx.x : 0;
  const int csv = g.col_start[c0 + cq], chv = g.col_h[c0 + cq];
  cplx<T> colv[zcols_per_thread<N>()];
  zcols_load<T, N>(Ts, g.ncols, c0, nc, colv);
  const cplx<T>* Xs = X ? X + (long)sys * ldx : nullptr;
  const cplx<T>* Es = E ? E + (long)sys * lde : nullptr;
  cplx<T>* Ys = Y + (long)sys * ldy;
  const cplx<T> sh = shift ? shift[sys] : cplx<T>{0, 0};
  const T ec = ecoef ? ecoef[sys] : T(0);
  const cplx<T>* Ps = DOT ? cd.p + (long)sys * cd.ldp : nullptr;
  // the pointwise operands of this thread's first points, loaded while the
  // columns are gathered and transformed (out-of-range slots load point run0)
  cplx<T> pf_p[KZ > 0 ? KZ : 1], pf_x[KZ > 0 ? KZ : 1], pf_e[KZ > 0 ? KZ : 1];
  T pf_k[KZ > 0 ? KZ : 1], pf_o[KZ > 0 ? KZ : 1];
#pragma unroll
  for (int k = 0; k < KZ; ++k) {
    const int i = run0 + threadIdx.x + k * 256;
    const int is = i < run1 ? i : run0;
    pf_p[k] = DOT ? Ps[is] : cplx<T>{0, 0};
    pf_x[k] = Xs ? Xs[is] : cplx<T>{0, 0};
    pf_k[k] = Xs ? static_cast<T>(g.kin[is]) : T(0);
    pf_e[k] = Es ? Es[is] : cplx<T>{0, 0};
    pf_o[k] = dout ? dout[is] : T(1);
  }
  put_tw<T, N>(tws, twv);
  if (threadIdx.x < nc) {
    cs[threadIdx.x] = csv;
    ch[threadIdx.x] = chv;
  }
  if (threadIdx.x == 0) cs[nc] = run1;
  zcols_store<T, N>(buf, nc, colv);
  __syncthreads();
  fft_lds<T, N, -1, 256, kZCols, false>(buf, tws, nc, [](int t, int e) { return t * LDZ + skew(e); });
  T pap = T(0);
  cplx<T> pc[8];
  if constexpr (PDOT) {
#pragma unroll
    for (int u = 0; u < 8; ++u) pc[u] = cplx<T>{0, 0};
  }
  // one point: y = scale FFT(...) [+ (kin - shift) x] [+ ec E], times dout
  auto point = [&](int i, cplx<T> pv, cplx<T> xv, T kn, cplx<T> ev, T dv) {
    int lo = 0, hi = nc;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (cs[mid] <= i) lo = mid; else hi = mid;
    }
    const int mz = i - cs[lo] - ch[lo];
    cplx<T> v = scale * buf[lo * LDZ + skew(mz < 0 ? mz + N : mz)];
    if (Xs) {
      const cplx<T> k = cplx<T>{kn - sh.x, -sh.y};
      v = v + k * xv;
    }
    if (Es) v = v + ec * ev;
    if (dout) v = dv * v;
    Ys[i] = v;
    if constexpr (DOT) pap += pv.x * v.x + pv.y * v.y;
    if constexpr (PDOT) {
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (u < pp.nv) pc[u] = pc[u] + cmulc(pp.Phi[(long)u * pp.ldphi + i], v);
    }
  };
#pragma unroll
  for (int k = 0; k < KZ; ++k) {
    const int i = run0 + threadIdx.x + k * 256;
    if (i < run1) point(i, pf_p[k], pf_x[k], pf_k[k], pf_e[k], pf_o[k]);
  }
  for (int i = run0 + threadIdx.x + KZ * 256; i < run1; i += 256)
    point(i, DOT ? Ps[i] : cplx<T>{0, 0}, Xs ? Xs[i] : cplx<T>{0, 0}, Xs ? static_cast<T>(g.kin[i]) : T(0),
          Es ? Es[i] : cplx<T>{0, 0}, dout ? dout[i] : T(1));
  if constexpr (PDOT) {
    // the workgroup's sums: over each wave by shuffles, then over the 4 waves
    __shared__ cplx<T> red[4][8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        pc[u].x += __shfl_xor(pc[u].x, o, 64);
        pc[u].y += __shfl_xor(pc[u].y, o, 64);
      }
    }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int u = 0; u < 8; ++u) red[threadIdx.x >> 6][u] = pc[u];
    }
    __syncthreads();
    if (threadIdx.x < 8)
      pp.part[((long)blockIdx.y * gridDim.x + blockIdx.x) * 8 + threadIdx.x] =
          (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
  }
  if constexpr (DOT) {
    __shared__ T smd[4];
    const T tot = zblock_sum(pap, smd);
    if (threadIdx.x == 0) {
      cd.part[(long)blockIdx.y * gridDim.x + blockIdx.x] = tot;
      if (blockIdx.x == 0) {
        const T th = cd.theta[sys];
        if (th >= T(0)) {
          cd.rr[sys] = th;
          cd.theta[sys] = T(-1);
        }
      }
    }
    if (cd.Cn && blockIdx.x == 0 && threadIdx.x < cd.nv)
      cd.Cp[(long)sys * cd.nv + threadIdx.x] = cd.Cn[(long)sys * cd.nv + threadIdx.x];
  }
}

// --------------------------------------------------------------- plane_hv
// One z plane of one system: x-inverse on the columns y that carry plane
// waves, y-filter on every row (inverse, times V, forward, with the middle
// stages fused in registers), x-forward on the same columns.  The first
// x-stage takes its butterflies straight from the plane's sphere columns
// (zero where the position map has none) and the last x-stage stores only the
// sphere columns back, so the plane is never cleared, scattered or gathered
// in LDS; the y-filter reads and writes only the 2 hy + 1 data rows at its
// ends.  Tile variants (chosen per grid, precision and batch size by the
// library's autotuner; the same transform, equal to rounding):
//   NT   threads per workgroup;
//   PAD  rows of N + 1 elements with the y-stages' threads on consecutive
//        rows (distinct LDS banks for every access), else rows of N
//        elements with consecutive butterflies of a row.
template <typename T, int N, int NT, bool PAD>
__global__ void __launch_bounds__(NT)
k_plane_hv(Geom g, const cplx<T>* __restrict__ tw, cplx<T>* __restrict__ Tb, long ldt,
           const T* __restrict__ Vt, const int* __restrict__ act) {
  constexpr int A = first_of(typename Plan<N>::type{});
  constexpr int B = second_of(typename Plan<N>::type{});
  constexpr int LD = PAD ? N + 1 : N;
  __shared__ cplx<T> pl[N * LD];
  __shared__ cplx<T> tws[N];
  const int z = blockIdx.x;
  const int sys = sys_of(act, blockIdx.y);
  cplx<T>* Ts = Tb + (long)sys * ldt + (long)z * g.ncols;
  const int* __restrict__ colof = g.col_of;
  const int hy = g.hy;
  const int ny = 2 * hy + 1;
  auto col = [hy](int t, int e) { return e * LD + pruned<N>(t, hy); };
  auto sphere_col = [colof, hy](int t, int e) { return colof[e * N + pruned<N>(t, hy)]; };
  // loads in the order they are needed: twiddles (first read after the first
  // stage's closing barrier), the first stage's column indices, the last
  // stage's (in flight while the transform runs), then the first stage's values
  const cplx<T> twv = get_tw<T, N>(tw);
  int cin[(N * (N / A) + NT - 1) / NT][A];
  stage_in_index<N, A, NT, N, true>(ny, sphere_col, cin);
  int cout[(N * (N / B) + NT - 1) / NT][B];
  stage_out_index<N, B, A, NT, N, true>(ny, sphere_col, cout);
  put_tw<T, N>(tws, twv);
  // x-inverse stage 1 (radix A, no twiddles) from the sphere columns
  fft_stage_gather<T, N, A, +1, NT, N, true>(ny, cin, Ts, [&](int t, int e, cplx<T> v) { pl[col(t, e)] = v; });
  // x-inverse stage 2 (radix B after A)
  fft_stage<T, N, B, A, +1, NT, N, true>(pl, tws, ny, col);
  const T* Vz = Vt + (long)z * N * N;
  fft_filter_rows_pruned<T, N, NT, N, PAD>(pl, tws, N, hy, [](int t, int e) { return t * LD + e; },
                                           [Vz](int t, int e) { return Vz[t * N + e]; });
  // x-forward stage 1
  fft_stage<T, N, A, 1, -1, NT, N, true>(pl, tws, ny, col);
  // x-forward stage 2, stored to the sphere columns
  fft_stage_scatter<T, N, B, A, -1, NT, N, true>(tws, ny, [&](int t, int e) { return pl[col(t, e)]; }, cout, Ts);
}

// --------------------------------------------------------- plane_pair_fwd
template <typename T, int N>
__global__ void __launch_bounds__(plane_threads<N>())
k_plane_pair_fwd(Geom g, const cplx<T>* __restrict__ tw, const cplx<T>* __restrict__ U, int nv,
                 const cplx<T>* __restrict__ X, long ldx, cplx<T>* __restrict__ Tb, long ldt) {
  constexpr int NT = plane_threads<N>();
  constexpr long NN = (long)N * N;
  __shared__ cplx<T> pl[N * N];
  __shared__ cplx<T> tws[N];
  const int z = blockIdx.x;
  const int s = blockIdx.y;           // s = j * nv + v
  const int j = s / nv, v = s - j * nv;
  const long n3 = NN * N;
  const cplx<T>* Uz = U + (long)v * n3 + z * NN;
  const cplx<T>* Xz = X + (long)j * ldx + z * NN;
  load_tw<T, N>(tws, tw);
  for (int i = threadIdx.x; i < N * N; i += NT) pl[i] = Uz[i] * Xz[i];
  __syncthreads();
  const int hy = g.hy;
  fft_lds<T, N, -1, NT, N, false>(pl, tws, N, [](int t, int e) { return t * N + e; });
  fft_lds<T, N, -1, NT, N, true>(pl, tws, 2 * hy + 1, [hy](int t, int e) { return e * N + pruned<N>(t, hy); });
  cplx<T>* Ts = Tb + (long)s * ldt + (long)z * g.ncols;
  for (int c = threadIdx.x; c < g.ncols; c += NT) Ts[c] = pl[g.col_pos[c]];
}

// --------------------------------------------------------------- plane_acc
template <typename T, int N>
__global__ void __launch_bounds__(plane_threads<N>())
k_plane_acc(Geom g, const cplx<T>* __restrict__ tw, const cplx<T>* __restrict__ Tb, long ldt,
            const cplx<T>* __restrict__ Psi, int nv, cplx<T>* __restrict__ out, long ldo, T coef,
            int accumulate) {
  constexpr int NT = plane_threads<N>();
  constexpr long NN = (long)N * N;
  constexpr int EPT = (N * N + NT - 1) / NT;
  __shared__ cplx<T> pl[N * N];
  __shared__ cplx<T> tws[N];
  const int z = blockIdx.x;
  const int j = blockIdx.y;
  const long n3 = NN * N;
  load_tw<T, N>(tws, tw);
  cplx<T> acc[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) acc[k] = cplx<T>{0, 0};
  const int hy = g.hy;
  for (int v = 0; v < nv; ++v) {
    for (int i = threadIdx.x; i < N * N; i += NT) pl[i] = cplx<T>{0, 0};
    __syncthreads();
    const cplx<T>* Ts = Tb + (long)(j * nv + v) * ldt + (long)z * g.ncols;
    for (int c = threadIdx.x; c < g.ncols; c += NT) pl[g.col_pos[c]] = Ts[c];
    __syncthreads();
    fft_lds<T, N, +1, NT, N, true>(pl, tws, 2 * hy + 1, [hy](int t, int e) { return e * N + pruned<N>(t, hy); });
    fft_lds<T, N, +1, NT, N, false>(pl, tws, N, [](int t, int e) { return t * N + e; });
    const cplx<T>* Pz = Psi + (long)v * n3 + z * NN;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int i = threadIdx.x + k * NT;
      if (i < N * N) acc[k] = acc[k] + Pz[i] * pl[i];
    }
    __syncthreads();
  }
  cplx<T>* Oz = out + (long)j * ldo + z * NN;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int i = threadIdx.x + k * NT;
    if (i < N * N) {
      cplx<T> r = coef * acc[k];
      if (accumulate) r = r + Oz[i];
      Oz[i] = r;
    }
  }
}

// -------------------------------------------------------------- plane_full
template <typename T, int N, int SIGN>
__global__ void __launch_bounds__(plane_threads<N>())
k_plane_full(const cplx<T>* __restrict__ tw, cplx<T>* G, long ldg, const cplx<T>* src) {
  constexpr int NT = plane_threads<N>();
  constexpr long NN = (long)N * N;
  __shared__ cplx<T> pl[N * N];
  __shared__ cplx<T> tws[N];
  cplx<T>* Gz = G + (long)blockIdx.y * ldg + blockIdx.x * NN;
  const cplx<T>* Sz = src ? src + (long)blockIdx.y * ldg + blockIdx.x * NN : Gz;
  load_tw<T, N>(tws, tw);
  for (int i = threadIdx.x; i < N * N; i += NT) pl[i] = Sz[i];
  __syncthreads();
  fft_lds<T, N, SIGN, NT, N, false>(pl, tws, N, [](int t, int e) { return t * N + e; });
  fft_lds<T, N, SIGN, NT, N, true>(pl, tws, N, [](int t, int e) { return e * N + t; });
  for (int i = threadIdx.x; i < N * N; i += NT) Gz[i] = pl[i];
}

// --------------------------------------------------------------- zfull_mul
template <typename T, int N>
__global__ void __launch_bounds__(256)
k_zfull_mul(const cplx<T>* __restrict__ tw, cplx<T>* __restrict__ G, long ldg,
            const T* __restrict__ mul, T scale) {
  constexpr int LDZ = skew(N) + 1;
  constexpr int NN = N * N;
  __shared__ cplx<T> buf[kZCols * LDZ];
  __shared__ cplx<T> tws[N];
  const int c0 = blockIdx.x * kZCols;
  const int nc = min(kZCols, NN - c0);
  cplx<T>* Gs = G + (long)blockIdx.y * ldg;
  const cplx<T> twv = get_tw<T, N>(tw);
  cplx<T> colv[zcols_per_thread<N>()];
  zcols_load<T, N>(Gs, NN, c0, nc, colv);
  put_tw<T, N>(tws, twv);
  zcols_store<T, N>(buf, nc, colv);
  __syncthreads();
  fft_lds<T, N, -1, 256, kZCols, false>(buf, tws, nc, [](int t, int e) { return t * LDZ + skew(e); });
  for (int i = threadIdx.x; i < N * nc; i += 256) {
    const int z = i / nc, cl = i - z * nc;
    buf[cl * LDZ + skew(z)] = (scale * mul[(long)z * NN + c0 + cl]) * buf[cl * LDZ + skew(z)];
  }
  __syncthreads();
  fft_lds<T, N, +1, 256, kZCols, false>(buf, tws, nc, [](int t, int e) { return t * LDZ + skew(e); });
  for (int i = threadIdx.x; i < N * nc; i += 256) {
    const int z = i / nc, cl = i - z * nc;
    Gs[(long)z * NN + c0 + cl] = buf[cl * LDZ + skew(z)];
  }
}

}  // namespace

bool grid_supported(int N) {
  switch (N) {
    case 16: case 24: case 32: case 40: case 48: case 64: case 72: return true;
    default: return false;
  }
}

#define LGW_DISPATCH_N(N, CALL)                 \
  switch (N) {                                  \
    case 16: { constexpr int NN_ = 16; CALL; } break; \
    case 24: { constexpr int NN_ = 24; CALL; } break; \
    case 32: { constexpr int NN_ = 32; CALL; } break; \
    case 40: { constexpr int NN_ = 40; CALL; } break; \
    case 48: { constexpr int NN_ = 48; CALL; } break; \
    case 64: { constexpr int NN_ = 64; CALL; } break; \
    case 72: { constexpr int NN_ = 72; CALL; } break; \
    default: break;                             \
  }

template <typename T>
void launch_zinv(const Geom& g, const cplx<T>* tw, const cplx<T>* X, long ldx, cplx<T>* Tb, long ldt,
                 T scale, const int* act, int nsys, hipStream_t s) {
  if (nsys <= 0) return;
  dim3 grid((g.ncols + kZCols - 1) / kZCols, nsys);
  LGW_DISPATCH_N(g.N, (k_zinv<T, NN_, false><<<grid, 256, 0, s>>>(g, tw, X, ldx, Tb, ldt, scale, act,
                                                                 ProjFeed<T>{}, nullptr)));
}

template <typename T>
void launch_zinv_fed(const Geom& g, const cplx<T>* tw, const ProjFeed<T>& f, const cplx<T>* D, cplx<T>* Xout,
                     long ldx, cplx<T>* Tb, long ldt, const int* act, int nsys, hipStream_t s) {
  if (nsys <= 0) return;
  dim3 grid((g.ncols + kZCols - 1) / kZCols, nsys);
  LGW_DISPATCH_N(g.N, (k_zinv<T, NN_, true><<<grid, 256, 0, s>>>(g, tw, D, ldx, Tb, ldt, T(1), act, f, Xout)));
}

// plane-pass tile variants: (threads, padded rows); grids of 64 and more take
// twice the threads (one workgroup per compute unit fits their planes)
template <int N, int V> constexpr int plane_var_threads() { return (N >= 64 ? 512 : 256) << (V >> 1); }

template <typename T, int N, int V>
void launch_plane_var(const Geom& g, const cplx<T>* tw, cplx<T>* Tb, long ldt, const T* Vt, const int* act,
                      int nsys, hipStream_t s) {
  constexpr int NT = plane_var_threads<N, V>();
  k_plane_hv<T, N, NT, (V & 1) != 0><<<dim3(g.N, nsys), NT, 0, s>>>(g, tw, Tb, ldt, Vt, act);
}

int plane_variants() { return 4; }

void plane_variant_shape(int N, int v, int* threads, int* pad) {
  *threads = (N >= 64 ? 512 : 256) << (v >> 1);
  *pad = v & 1;
}

template <typename T>
void launch_plane_hv(const Geom& g, const cplx<T>* tw, cplx<T>* Tb, long ldt, const T* Vt,
                     const int* act, int nsys, hipStream_t s, int variant) {
  if (nsys <= 0) return;
  switch (variant & 3) {
    case 0: LGW_DISPATCH_N(g.N, (launch_plane_var<T, NN_, 0>(g, tw, Tb, ldt, Vt, act, nsys, s))); break;
    case 1: LGW_DISPATCH_N(g.N, (launch_plane_var<T, NN_, 1>(g, tw, Tb, ldt, Vt, act, nsys, s))); break;
    case 2: LGW_DISPATCH_N(g.N, (launch_plane_var<T, NN_, 2>(g, tw, Tb, ldt, Vt, act, nsys, s))); break;
    default: LGW_DISPATCH_N(g.N, (launch_plane_var<T, NN_, 3>(g, tw, Tb, ldt, Vt, act, nsys, s))); break;
  }
}

template <typename T>
void launch_zfwd(const Geom& g, const cplx<T>* tw, const cplx<T>* Tb, long ldt, T scale,
                 const cplx<T>* X, long ldx, const cplx<T>* shift, const cplx<T>* E, long lde,
                 const T* ecoef, cplx<T>* Y, long ldy, const int* act, int nsys, hipStream_t s,
                 const T* dout, const CgDot<T>& cd, const ProjPart<T>* pp) {
  if (nsys <= 0) return;
  dim3 grid(zcol_blocks(g), nsys);
  const ProjPart<T> pq = pp ? *pp : ProjPart<T>{};
  if (cd.part) {
    LGW_DISPATCH_N(g.N, (k_zfwd<T, NN_, 1><<<grid, 256, 0, s>>>(g, tw, Tb, ldt, scale, X, ldx, shift, E, lde,
                                                              ecoef, Y, ldy, act, dout, cd, pq)));
  } else if (pq.part) {
    LGW_DISPATCH_N(g.N, (k_zfwd<T, NN_, 2><<<grid, 256, 0, s>>>(g, tw, Tb, ldt, scale, X, ldx, shift, E, lde,
                                                              ecoef, Y, ldy, act, dout, cd, pq)));
  } else {
    LGW_DISPATCH_N(g.N, (k_zfwd<T, NN_, 0><<<grid, 256, 0, s>>>(g, tw, Tb, ldt, scale, X, ldx, shift, E, lde,
                                                              ecoef, Y, ldy, act, dout, cd, pq)));
  }
}

int zcol_blocks(const Geom& g) { return (g.ncols + kZCols - 1) / kZCols; }

template <typename T>
void launch_plane_pair_fwd(const Geom& g, const cplx<T>* tw, const cplx<T>* U, int nv, const cplx<T>* X,
                           long ldx, int nj, cplx<T>* Tb, long ldt, hipStream_t s) {
  if (nj <= 0) return;
  dim3 grid(g.N, nj * nv);
  LGW_DISPATCH_N(g.N, (k_plane_pair_fwd<T, NN_><<<grid, plane_threads<NN_>(), 0, s>>>(g, tw, U, nv, X, ldx, Tb, ldt)));
}

template <typename T>
void launch_plane_acc(const Geom& g, const cplx<T>* tw, const cplx<T>* Tb, long ldt, const cplx<T>* Psi,
                      int nv, cplx<T>* out, long ldo, T coef, int nj, bool accumulate, hipStream_t s) {
  if (nj <= 0) return;
  dim3 grid(g.N, nj);
  LGW_DISPATCH_N(g.N, (k_plane_acc<T, NN_><<<grid, plane_threads<NN_>(), 0, s>>>(g, tw, Tb, ldt, Psi, nv, out, ldo,
                                                                              coef, accumulate ? 1 : 0)));
}

template <typename T>
void launch_plane_full(int N, const cplx<T>* tw, cplx<T>* G, long ldg, int nvec, int sign, hipStream_t s,
                       const cplx<T>* src) {
  if (nvec <= 0) return;
  dim3 grid(N, nvec);
  if (sign < 0) {
    LGW_DISPATCH_N(N, (k_plane_full<T, NN_, -1><<<grid, plane_threads<NN_>(), 0, s>>>(tw, G, ldg, src)));
  } else {
    LGW_DISPATCH_N(N, (k_plane_full<T, NN_, +1><<<grid, plane_threads<NN_>(), 0, s>>>(tw, G, ldg, src)));
  }
}

template <typename T>
void launch_zfull_mul(int N, const cplx<T>* tw, cplx<T>* G, long ldg, const T* mul, T scale, int nvec,
                      hipStream_t s) {
  if (nvec <= 0) return;
  dim3 grid((N * N + kZCols - 1) / kZCols, nvec);
  LGW_DISPATCH_N(N, (k_zfull_mul<T, NN_><<<grid, 256, 0, s>>>(tw, G, ldg, mul, scale)));
}

#define LGW_INST(T)                                                                                   \
  template void launch_zinv<T>(const Geom&, const cplx<T>*, const cplx<T>*, long, cplx<T>*, long, T,  \
                               const int*, int, hipStream_t);                                         \
  template void launch_zinv_fed<T>(const Geom&, const cplx<T>*, const ProjFeed<T>&, const cplx<T>*,    \
                                   cplx<T>*, long, cplx<T>*, long, const int*, int, hipStream_t);     \
  template void launch_plane_hv<T>(const Geom&, const cplx<T>*, cplx<T>*, long, const T*, const int*, \
                                   int, hipStream_t, int);                                            \
  template void launch_zfwd<T>(const Geom&, const cplx<T>*, const cplx<T>*, long, T, const cplx<T>*,  \
                               long, const cplx<T>*, const cplx<T>*, long, const T*, cplx<T>*, long,  \
                               const int*, int, hipStream_t, const T*, const CgDot<T>&,               \
                               const ProjPart<T>*);                                                   \
  template void launch_plane_pair_fwd<T>(const Geom&, const cplx<T>*, const cplx<T>*, int,            \
                                         const cplx<T>*, long, int, cplx<T>*, long, hipStream_t);     \
  template void launch_plane_acc<T>(const Geom&, const cplx<T>*, const cplx<T>*, long, const cplx<T>*, \
                                    int, cplx<T>*, long, T, int, bool, hipStream_t);                  \
  template void launch_plane_full<T>(int, const cplx<T>*, cplx<T>*, long, int, int, hipStream_t,       \
                                     const cplx<T>*);                                                 \
  template void launch_zfull_mul<T>(int, const cplx<T>*, cplx<T>*, long, const T*, T, int, hipStream_t);

LGW_INST(double)
LGW_INST(float)

}  // namespace lgw
