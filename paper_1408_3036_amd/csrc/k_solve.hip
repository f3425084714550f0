// Projector, batched CG / SQMR updates, residuals, Lanczos BLAS-1 and layout
// kernels (gfx950).  One workgroup owns one system in the per-system kernels:
// its reductions are exact block reductions in a fixed order (deterministic).
#include "kernels.h"

namespace lgw {

namespace {

constexpr int NT = 256;

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum K values over the workgroup; every thread gets the totals in v[].
template <typename T, int K>
__device__ __forceinline__ void block_sum(T (&v)[K], T* sm /* >= K*NT/64 */) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    T s = wave_sum(v[k]);
    if (lane == 0) sm[k * (NT / 64) + w] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    T s = T(0);
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += sm[k * (NT / 64) + i];
    v[k] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- projector
template <typename T>
__global__ void __launch_bounds__(NT)
k_proj(const cplx<T>* __restrict__ Phi, long ldphi, int nv, int npw, cplx<T>* __restrict__ Y,
       long ldy, const int* __restrict__ act) {
  constexpr int VB = 8;
  __shared__ T sm[2 * VB * (NT / 64)];
  __shared__ cplx<T> c[kMaxBands];
  const int sys = sys_of(act, blockIdx.x);
  cplx<T>* Ys = Y + (long)sys * ldy;
  for (int v0 = 0; v0 < nv; v0 += VB) {
    T acc[2 * VB];
#pragma unroll
    for (int u = 0; u < 2 * VB; ++u) acc[u] = T(0);
    for (int i = threadIdx.x; i < npw; i += NT) {
      const cplx<T> y = Ys[i];
#pragma unroll
      for (int u = 0; u < VB; ++u) {
        if (v0 + u < nv) {
          const cplx<T> p = Phi[(long)(v0 + u) * ldphi + i];
          acc[2 * u] += p.x * y.x + p.y * y.y;
          acc[2 * u + 1] += p.x * y.y - p.y * y.x;
        }
      }
    }
    block_sum<T, 2 * VB>(acc, sm);
    if (threadIdx.x == 0) {
      for (int u = 0; u < VB && v0 + u < nv; ++u) c[v0 + u] = cplx<T>{acc[2 * u], acc[2 * u + 1]};
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < npw; i += NT) {
    cplx<T> y = Ys[i];
    for (int v = 0; v < nv; ++v) y = y - c[v] * Phi[(long)v * ldphi + i];
    Ys[i] = y;
  }
}

// ---------------------------------------------------------------- CG
// Projector partial sums left for the next operator application (ProjFeed):
// acc[2u], acc[2u+1] += conj(Phi_{v0+u}[i]) (pre[i] y) for the bands
// v0 + u < nv of one group of eight
template <typename T>
__device__ __forceinline__ void feed_acc(const ProjFeed<T>& f, int v0, int i, cplx<T> y, T (&acc)[16]) {
  if (f.pre) y = f.pre[i] * y;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    if (v0 + u < f.nv) {
      const cplx<T> ph = f.Phi[(long)(v0 + u) * f.ldphi + i];
      acc[2 * u] += ph.x * y.x + ph.y * y.y;
      acc[2 * u + 1] += ph.x * y.y - ph.y * y.x;
    }
  }
}
// Workgroup sums of the 16 values of a group, stored to slice k of system
// sys.  Within a wave the values are halved at each exchange (each lane keeps
// one half and adds its partner's copy of it: 8 + 4 + 2 + 1 shuffles leave one
// value per lane, summed over 16 lanes; two more finish the wave); the waves'
// totals meet in LDS.  Fixed order, so every call sums alike.
// one halving exchange at lane distance 4H: lanes keep H values
// (compile-time H, so that every index into acc is static)
template <typename T, int H>
__device__ __forceinline__ void feed_halve(T (&acc)[16], int lane, int& base) {
  constexpr int O = 4 * H;
  const bool up = (lane & O) != 0;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const T send = up ? acc[j] : acc[j + H];
    const T keep = up ? acc[j + H] : acc[j];
    acc[j] = keep + __shfl_xor(send, O, 64);
  }
  base += up ? H : 0;
}
template <typename T>
__device__ __forceinline__ void feed_store(const ProjFeed<T>& f, int v0, int k, int sys, T (&acc)[16], T* sm) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int base = 0;
  feed_halve<T, 8>(acc, lane, base);
  feed_halve<T, 4>(acc, lane, base);
  feed_halve<T, 2>(acc, lane, base);
  feed_halve<T, 1>(acc, lane, base);
  acc[0] += __shfl_xor(acc[0], 2, 64);
  acc[0] += __shfl_xor(acc[0], 1, 64);
  if ((lane & 3) == 0) sm[w * 16 + base] = acc[0];
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 16 && v0 + t / 2 < f.nv) {
    T tot = T(0);
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) tot += sm[i * 16 + t];
    T* P = reinterpret_cast<T*>(f.part + ((long)k * f.ntot + sys) * f.nv + v0);
    P[t] = tot;
  }
  __syncthreads();
}
template <typename T>
__device__ __forceinline__ void feed_zero(T (&acc)[16]) {
#pragma unroll
  for (int u = 0; u < 16; ++u) acc[u] = T(0);
}

template <typename T>
__global__ void __launch_bounds__(NT)
k_cg_init(SolveVecs<T> v, const cplx<T>* __restrict__ b, long ldb, const int* __restrict__ bidx,
          int npw, int keep_x, const int* __restrict__ act) {
  __shared__ T sm[NT / 64];
  const int sys = sys_of(act, blockIdx.x);
  const cplx<T>* bs = b + (long)(bidx ? bidx[sys] : sys) * ldb;
  cplx<T>* x = v.x + (long)sys * v.ld;
  cplx<T>* r = v.r + (long)sys * v.ld;
  cplx<T>* p = v.p + (long)sys * v.ld;
  T acc[1] = {T(0)};
  for (int i = threadIdx.x; i < npw; i += NT) {
    const cplx<T> bi = bs[i];
    if (!keep_x) x[i] = cplx<T>{0, 0};
    r[i] = bi;
    p[i] = bi;
    acc[0] += norm2(bi);
  }
  block_sum<T, 1>(acc, sm);
  if (threadIdx.x == 0) {
    v.rr[sys] = acc[0];
    v.theta[sys] = T(-1);
    if (!keep_x) { v.bb[sys] = acc[0]; v.iters[sys] = 0; }
    v.flag[sys] = acc[0] == T(0) ? FLAG_CONV : 0;
  }
}

// Initialisation of a small preconditioned CG batch over the split grid
// (nsplit, nsys): x = 0 (unless kept), r = p = b on each slice, the slice sums
// conj(Phi_v) (pre .* b) for the first projection, and |b|^2 through the
// ticket (the last workgroup of a system sums the slice norms in one wave and
// writes rr, theta, bb, the count and the flag; the counters are zero
// between launches).
template <typename T>
__global__ void __launch_bounds__(NT)
k_cg_init_fed(SolveVecs<T> v, const cplx<T>* __restrict__ b, long ldb, const int* __restrict__ bidx, int npw,
              int keep_x, const int* __restrict__ act, T* __restrict__ npart, ProjFeed<T> f) {
  __shared__ T sm[16 * (NT / 64)];
  __shared__ int last;
  const int slot = blockIdx.y;
  const int sys = sys_of(act, slot);
  const int nsplit = f.nsplit;
  const cplx<T>* bs = b + (long)(bidx ? bidx[sys] : sys) * ldb;
  const int chunk = (npw + nsplit - 1) / nsplit;
  const int i0 = blockIdx.x * chunk, i1 = min(npw, i0 + chunk);
  const long off = (long)sys * v.ld;
  cplx<T>* x = v.x + off;
  cplx<T>* r = v.r + off;
  cplx<T>* p = v.p + off;
  T acc[1] = {T(0)};
  T fa[16];
  feed_zero(fa);
  for (int i = i0 + threadIdx.x; i < i1; i += NT) {
    const cplx<T> bi = bs[i];
    cplx<T> ph[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) ph[u] = u < f.nv ? f.Phi[(long)u * f.ldphi + i] : cplx<T>{0, 0};
    const T sc = f.pre ? f.pre[i] : T(1);
    if (!keep_x) x[i] = cplx<T>{0, 0};
    r[i] = bi;
    p[i] = bi;
    acc[0] += norm2(bi);
    const cplx<T> y = sc * bi;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      fa[2 * u] += ph[u].x * y.x + ph[u].y * y.y;
      fa[2 * u + 1] += ph[u].x * y.y - ph[u].y * y.x;
    }
  }
  block_sum<T, 1>(acc, sm);
  feed_store(f, 0, blockIdx.x, sys, fa, sm);
  for (int v0 = 8; v0 < f.nv; v0 += 8) {
    feed_zero(fa);
    for (int i = i0 + threadIdx.x; i < i1; i += NT) feed_acc(f, v0, i, bs[i], fa);
    feed_store(f, v0, blockIdx.x, sys, fa, sm);
  }
  if (threadIdx.x == 0) {
    npart[(long)slot * nsplit + blockIdx.x] = acc[0];
    const int ticket = __hip_atomic_fetch_add(v.cnt + slot, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = ticket == nsplit - 1;
  }
  __syncthreads();
  if (!last || threadIdx.x >= 64) return;
  const T e = threadIdx.x < nsplit
                  ? __hip_atomic_load(npart + (long)slot * nsplit + threadIdx.x, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT)
                  : T(0);
  const T bb = wave_sum(e);
  if (threadIdx.x != 0) return;
  v.cnt[slot] = 0;
  v.rr[sys] = bb;
  v.theta[sys] = T(-1);
  if (!keep_x) {
    v.bb[sys] = bb;
    v.iters[sys] = 0;
  }
  v.flag[sys] = bb == T(0) ? FLAG_CONV : 0;
}

template <typename T>
__global__ void __launch_bounds__(NT)
k_cg_step(SolveVecs<T> v, int npw, T tol2, const int* __restrict__ act) {
  __shared__ T sm[NT / 64];
  const int sys = sys_of(act, blockIdx.x);
  if (v.flag[sys]) return;
  cplx<T>* x = v.x + (long)sys * v.ld;
  cplx<T>* r = v.r + (long)sys * v.ld;
  cplx<T>* p = v.p + (long)sys * v.ld;
  const cplx<T>* Ap = v.Ap + (long)sys * v.ld;
  T acc[1] = {T(0)};
  for (int i = threadIdx.x; i < npw; i += NT) {
    const cplx<T> a = p[i], b = Ap[i];
    acc[0] += a.x * b.x + a.y * b.y;
  }
  block_sum<T, 1>(acc, sm);
  const T pAp = acc[0];
  const T parked = v.theta[sys];
  const T rr = parked >= T(0) ? parked : v.rr[sys];
  if (!(pAp > T(0))) {
    if (threadIdx.x == 0) v.flag[sys] = FLAG_BREAK;
    return;
  }
  const T alpha = rr / pAp;
  acc[0] = T(0);
  for (int i = threadIdx.x; i < npw; i += NT) {
    const cplx<T> pi = p[i];
    x[i] = x[i] + alpha * pi;
    const cplx<T> ri = r[i] - alpha * Ap[i];
    r[i] = ri;
    acc[0] += norm2(ri);
  }
  block_sum<T, 1>(acc, sm);
  const T rrn = acc[0];
  const T beta = rrn / rr;
  for (int i = threadIdx.x; i < npw; i += NT) p[i] = r[i] + beta * p[i];
  if (threadIdx.x == 0) {
    v.rr[sys] = rrn;
    v.theta[sys] = T(-1);
    v.iters[sys] += 1;
    if (rrn <= tol2 * v.bb[sys]) v.flag[sys] = FLAG_CONV;
  }
}

// ---------------------------------------------------------------- SQMR
// Symmetric QMR without look-ahead for the complex-symmetric projected
// systems, with the bilinear form (a, b)_J = sum_i a[npw-1-i] b[i] (the
// unconjugated grid product: index npw-1-i holds -m).
template <typename T>
__global__ void __launch_bounds__(NT)
k_sqmr_init(SolveVecs<T> v, const cplx<T>* __restrict__ b, long ldb, const int* __restrict__ bidx,
            int npw, int keep_x, const int* __restrict__ act) {
  __shared__ T sm[3 * (NT / 64)];
  const int sys = sys_of(act, blockIdx.x);
  const cplx<T>* bs = b + (long)(bidx ? bidx[sys] : sys) * ldb;
  cplx<T>* x = v.x + (long)sys * v.ld;
  cplx<T>* r = v.r + (long)sys * v.ld;
  cplx<T>* q = v.p + (long)sys * v.ld;
  cplx<T>* d = v.d + (long)sys * v.ld;
  T acc[3] = {T(0), T(0), T(0)};
  for (int i = threadIdx.x; i < npw; i += NT) {
    const cplx<T> bi = bs[i];
    const cplx<T> bj = bs[npw - 1 - i];
    if (!keep_x) x[i] = cplx<T>{0, 0};
    d[i] = cplx<T>{0, 0};
    r[i] = bi;
    q[i] = bi;
    acc[0] += norm2(bi);
    const cplx<T> pr = bi * bj;
    acc[1] += pr.x;
    acc[2] += pr.y;
  }
  block_sum<T, 3>(acc, sm);
  if (threadIdx.x == 0) {
    const T nb = sqrt(acc[0]);
    v.rr[sys] = nb;                 // tau
    v.theta[sys] = T(0);
    v.rho[sys] = cplx<T>{acc[1], acc[2]};
    if (!keep_x) { v.bb[sys] = acc[0]; v.iters[sys] = 0; }
    v.flag[sys] = acc[0] == T(0) ? FLAG_CONV : 0;
  }
}

template <typename T>
__global__ void __launch_bounds__(NT)
k_sqmr_step(SolveVecs<T> v, int npw, T tol, const int* __restrict__ act) {
  __shared__ T sm[3 * (NT / 64)];
  const int sys = sys_of(act, blockIdx.x);
  if (v.flag[sys]) return;
  cplx<T>* x = v.x + (long)sys * v.ld;
  cplx<T>* r = v.r + (long)sys * v.ld;
  cplx<T>* q = v.p + (long)sys * v.ld;
  cplx<T>* d = v.d + (long)sys * v.ld;
  const cplx<T>* t = v.Ap + (long)sys * v.ld;
  // sigma = (q, t)_J
  T acc[3] = {T(0), T(0), T(0)};
  for (int i = threadIdx.x; i < npw; i += NT) {
    const cplx<T> pr = q[npw - 1 - i] * t[i];
    acc[0] += pr.x;
    acc[1] += pr.y;
  }
  {
    T a2[2] = {acc[0], acc[1]};
    block_sum<T, 2>(a2, sm);
    acc[0] = a2[0];
    acc[1] = a2[1];
  }
  const cplx<T> sigma = cplx<T>{acc[0], acc[1]};
  const cplx<T> rho = v.rho[sys];
  const T sn = norm2(sigma);
  if (!(sn > T(0))) {
    if (threadIdx.x == 0) v.flag[sys] = FLAG_BREAK;
    return;
  }
  // alpha = rho / sigma
  const cplx<T> alpha = cplx<T>{(rho.x * sigma.x + rho.y * sigma.y) / sn,
                                (rho.y * sigma.x - rho.x * sigma.y) / sn};
  // r -= alpha t on the pairs (i, npw-1-i); accumulate |r|^2 and (r, r)_J
  acc[0] = acc[1] = acc[2] = T(0);
  const int half = (npw + 1) / 2;
  for (int i = threadIdx.x; i < half; i += NT) {
    const int j = npw - 1 - i;
    const cplx<T> ri = r[i] - alpha * t[i];
    r[i] = ri;
    if (j != i) {
      const cplx<T> rj = r[j] - alpha * t[j];
      r[j] = rj;
      acc[0] += norm2(ri) + norm2(rj);
      const cplx<T> pr = ri * rj;
      acc[1] += T(2) * pr.x;
      acc[2] += T(2) * pr.y;
    } else {
      acc[0] += norm2(ri);
      const cplx<T> pr = ri * ri;
      acc[1] += pr.x;
      acc[2] += pr.y;
    }
  }
  block_sum<T, 3>(acc, sm);
  const T tau = v.rr[sys];
  const T th_old = v.theta[sys];
  const T th = sqrt(acc[0]) / tau;
  const T c2 = T(1) / (T(1) + th * th);
  const T tau_n = tau * th * sqrt(c2);
  const cplx<T> rho_n = cplx<T>{acc[1], acc[2]};
  const T rn = norm2(rho);
  const cplx<T> beta = cplx<T>{(rho_n.x * rho.x + rho_n.y * rho.y) / rn,
                               (rho_n.y * rho.x - rho_n.x * rho.y) / rn};
  const T f1 = c2 * th_old * th_old;
  const cplx<T> f2 = c2 * alpha;
  for (int i = threadIdx.x; i < npw; i += NT) {
    const cplx<T> qi = q[i];
    const cplx<T> di = f1 * d[i] + f2 * qi;
    d[i] = di;
    x[i] = x[i] + di;
    q[i] = r[i] + beta * qi;
  }
  if (threadIdx.x == 0) {
    const int it = v.iters[sys] + 1;
    v.iters[sys] = it;
    v.rr[sys] = tau_n;
    v.theta[sys] = th;
    v.rho[sys] = rho_n;
    // quasi-residual test (|r_n| <= sqrt(n+1) tau_n is the worst case; the true
    // residual is checked on the host after every solve)
    if (tau_n <= tol * sqrt(v.bb[sys])) v.flag[sys] = FLAG_CONV;
    else if (!(norm2(rho_n) > T(0))) v.flag[sys] = FLAG_BREAK;
  }
}

// ---------------------------------------------------------------- residual
template <typename T>
__global__ void __launch_bounds__(NT)
k_resid(const cplx<T>* __restrict__ b, long ldb, const int* __restrict__ bidx,
        const cplx<T>* __restrict__ AX, long lda, cplx<T>* __restrict__ R, long ldr,
        double* __restrict__ res, int npw, const int* __restrict__ act) {
  __shared__ double sm[NT / 64];
  const int sys = sys_of(act, blockIdx.x);
  const cplx<T>* bs = b + (long)(bidx ? bidx[sys] : sys) * ldb;
  const cplx<T>* as = AX + (long)sys * lda;
  cplx<T>* rs = R ? R + (long)sys * ldr : nullptr;
  double acc[1] = {0.0};
  for (int i = threadIdx.x; i < npw; i += NT) {
    const cplx<T> ri = bs[i] - as[i];
    if (rs) rs[i] = ri;
    acc[0] += (double)norm2(ri);
  }
  block_sum<double, 1>(acc, sm);
  if (threadIdx.x == 0) res[sys] = acc[0];
}

// the same over ns workgroups per system (grid (ns, nsys)): res[sys][blk] are
// the slice norms, summed by the caller; AX null stands for zero (R = b)
template <typename T>
__global__ void __launch_bounds__(NT)
k_resid_split(const cplx<T>* __restrict__ b, long ldb, const int* __restrict__ bidx,
              const cplx<T>* __restrict__ AX, long lda, cplx<T>* __restrict__ R, long ldr,
              double* __restrict__ res, int npw, const int* __restrict__ act) {
  __shared__ double sm[NT / 64];
  const int sys = sys_of(act, blockIdx.y);
  const int chunk = (npw + gridDim.x - 1) / gridDim.x;
  const int i0 = blockIdx.x * chunk, i1 = min(npw, i0 + chunk);
  const cplx<T>* bs = b + (long)(bidx ? bidx[sys] : sys) * ldb;
  const cplx<T>* as = AX ? AX + (long)sys * lda : nullptr;
  cplx<T>* rs = R ? R + (long)sys * ldr : nullptr;
  double acc[1] = {0.0};
  for (int i = i0 + threadIdx.x; i < i1; i += NT) {
    const cplx<T> ri = as ? bs[i] - as[i] : bs[i];
    if (rs) rs[i] = ri;
    acc[0] += (double)norm2(ri);
  }
  block_sum<double, 1>(acc, sm);
  if (threadIdx.x == 0) res[(long)sys * gridDim.x + blockIdx.x] = acc[0];
}

// ---------------------------------------------------------------- BLAS-1
constexpr int kDotBlocks = 64;

// partial[i][blk] = sum over the block's share of conj(A_i) w
__global__ void __launch_bounds__(NT)
k_dots_partial(const z64* __restrict__ A, long lda, const z64* __restrict__ w, long n,
               z64* __restrict__ partial) {
  __shared__ double sm[2 * (NT / 64)];
  const int i = blockIdx.y;
  const z64* a = A + (long)i * lda;
  double acc[2] = {0.0, 0.0};
  for (long e = (long)blockIdx.x * NT + threadIdx.x; e < n; e += (long)gridDim.x * NT) {
    const z64 p = cmulc(a[e], w[e]);
    acc[0] += p.x;
    acc[1] += p.y;
  }
  block_sum<double, 2>(acc, sm);
  if (threadIdx.x == 0) partial[(long)i * gridDim.x + blockIdx.x] = z64{acc[0], acc[1]};
}

__global__ void k_dots_final(const z64* __restrict__ partial, int nblk, z64* __restrict__ h) {
  const int i = blockIdx.x;
  if (threadIdx.x == 0) {
    z64 s{0, 0};
    for (int b = 0; b < nblk; ++b) s = s + partial[(long)i * nblk + b];
    h[i] = s;
  }
}

// One classical Gram-Schmidt pass after k_dots_partial: h_i = sum_b
// partial[i][b] (summed in order by every workgroup, as k_dots_final does),
// w = in - sum_i h_i A_i with in = src or w; workgroup 0 stores Re h_{m-1}
// in re_last when given.  m <= kCgsMax.
constexpr int kCgsMax = 512;
__global__ void __launch_bounds__(NT)
k_cgs_sub(const z64* __restrict__ A, long lda, int m, const z64* __restrict__ partial, int nblk, z64* w,
          const z64* src, long n, double* __restrict__ re_last) {
  __shared__ z64 hs[kCgsMax];
  for (int i = threadIdx.x; i < m; i += NT) {
    z64 s{0, 0};
    for (int b = 0; b < nblk; ++b) s = s + partial[(long)i * nblk + b];
    hs[i] = s;
  }
  __syncthreads();
  if (re_last && blockIdx.x == 0 && threadIdx.x == 0) *re_last = hs[m - 1].x;
  const z64* in = src ? src : w;
  for (long e = (long)blockIdx.x * NT + threadIdx.x; e < n; e += (long)gridDim.x * NT) {
    z64 acc = in[e];
    for (int i = 0; i < m; ++i) acc = acc - hs[i] * A[(long)i * lda + e];
    w[e] = acc;
  }
}

__global__ void __launch_bounds__(NT) k_copy(const z64* __restrict__ a, z64* __restrict__ b, long n) {
  for (long e = (long)blockIdx.x * NT + threadIdx.x; e < n; e += (long)gridDim.x * NT) b[e] = a[e];
}

__global__ void k_re_of(const z64* __restrict__ h, double* __restrict__ out) {
  if (threadIdx.x == 0) *out = h->x;
}

__global__ void __launch_bounds__(NT)
k_gemv_sub(const z64* __restrict__ A, long lda, int m, const z64* __restrict__ h,
           z64* __restrict__ w, long n) {
  for (long e = (long)blockIdx.x * NT + threadIdx.x; e < n; e += (long)gridDim.x * NT) {
    z64 acc = w[e];
    for (int i = 0; i < m; ++i) acc = acc - h[i] * A[(long)i * lda + e];
    w[e] = acc;
  }
}

__global__ void k_alpha_final(const z64* __restrict__ partial, int nblk, double* __restrict__ alpha) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[b].x;
    *alpha = s;
  }
}

__global__ void __launch_bounds__(NT)
k_lanczos_sub(z64* w, const z64* __restrict__ q, const z64* __restrict__ qprev,
              const double* __restrict__ alpha, const double* __restrict__ beta_prev, long n, const z64* src) {
  const double a = *alpha;
  const double b = beta_prev ? *beta_prev : 0.0;
  const z64* in = src ? src : w;
  for (long e = (long)blockIdx.x * NT + threadIdx.x; e < n; e += (long)gridDim.x * NT) {
    z64 r = in[e] - a * q[e];
    if (qprev) r = r - b * qprev[e];
    w[e] = r;
  }
}

// *out = the norm; with pair, also pair[0] = *alpha and pair[1] = the norm
// (a Lanczos step's two scalars side by side for one readback)
__global__ void k_norm_final(const z64* __restrict__ partial, int nblk, double* __restrict__ out,
                             const double* __restrict__ alpha, double* __restrict__ pair) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[b].x;
    *out = sqrt(s);
    if (pair) {
      pair[0] = *alpha;
      pair[1] = sqrt(s);
    }
  }
}

__global__ void __launch_bounds__(NT)
k_scale_into(const z64* __restrict__ w, const double* __restrict__ nrm, z64* __restrict__ q, long n) {
  const double s = 1.0 / *nrm;
  for (long e = (long)blockIdx.x * NT + threadIdx.x; e < n; e += (long)gridDim.x * NT) q[e] = s * w[e];
}

__global__ void __launch_bounds__(NT)
k_axpby(z64* __restrict__ y, const z64* __restrict__ x, z64 a, z64 b, long n) {
  for (long e = (long)blockIdx.x * NT + threadIdx.x; e < n; e += (long)gridDim.x * NT)
    y[e] = a * x[e] + b * y[e];
}

__global__ void __launch_bounds__(NT)
k_add(z64* __restrict__ y, const z64* __restrict__ a, const z64* __restrict__ b, long n) {
  for (long e = (long)blockIdx.x * NT + threadIdx.x; e < n; e += (long)gridDim.x * NT) y[e] = a[e] + b[e];
}

__global__ void __launch_bounds__(NT)
k_finite(const double* __restrict__ x, long n, int* __restrict__ flag) {
  bool bad = false;
  for (long e = (long)blockIdx.x * NT + threadIdx.x; e < n; e += (long)gridDim.x * NT)
    bad |= !isfinite(x[e]);
  if (bad) atomicOr(flag, 1);
}

__global__ void __launch_bounds__(NT)
k_cvt_64_32(const z64* __restrict__ in, z32* __restrict__ out, long n) {
  for (long e = (long)blockIdx.x * NT + threadIdx.x; e < n; e += (long)gridDim.x * NT)
    out[e] = cvt<float>(in[e]);
}

__global__ void __launch_bounds__(NT)
k_cvt_32_64(const z32* __restrict__ in, z64* __restrict__ out, long n) {
  for (long e = (long)blockIdx.x * NT + threadIdx.x; e < n; e += (long)gridDim.x * NT)
    out[e] = cvt<double>(in[e]);
}

__global__ void __launch_bounds__(NT)
k_mul(z64* __restrict__ y, const z64* __restrict__ a, const z64* __restrict__ b, long n) {
  for (long e = (long)blockIdx.x * NT + threadIdx.x; e < n; e += (long)gridDim.x * NT) y[e] = a[e] * b[e];
}

template <class T>
__global__ void __launch_bounds__(NT)
k_fill(cplx<T>* __restrict__ p, cplx<T> v, long n) {
  for (long e = (long)blockIdx.x * NT + threadIdx.x; e < n; e += (long)gridDim.x * NT) p[e] = v;
}

// x[sys] += scale[sys] * (d .* e[sys]) (e in single precision; d optional,
// applied in single precision); assign: x[sys] = scale[sys] * (d .* e[sys])
__global__ void __launch_bounds__(NT)
k_cvt_32_64_axpy(const z32* __restrict__ e, z64* __restrict__ x, const double* __restrict__ scale,
                 const int* __restrict__ act, long ld, int npw, const float* __restrict__ d, int assign) {
  const int sys = sys_of(act, blockIdx.y);
  const double s = scale[sys];
  for (int i = blockIdx.x * NT + threadIdx.x; i < npw; i += gridDim.x * NT) {
    const z32 e32 = e[(long)sys * ld + i];
    const z64 ev = cvt<double>(d ? d[i] * e32 : e32);
    x[(long)sys * ld + i] = assign ? s * ev : x[(long)sys * ld + i] + s * ev;
  }
}

// ------------------------------------------------------------- transposes
// [v][a][b] -> [v][b][a] with a = N*N (x,y), b = N (z); 32x32 LDS tiles.
template <bool CONJ>
__global__ void __launch_bounds__(NT)
k_transpose(const z64* __restrict__ in, long ldi, z64* __restrict__ out, long ldo, int A, int B) {
  __shared__ z64 tile[32][33];
  const z64* src = in + (long)blockIdx.z * ldi;
  z64* dst = out + (long)blockIdx.z * ldo;
  const int a0 = blockIdx.x * 32, b0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int a = a0 + k, b = b0 + tx;
    if (a < A && b < B) {
      z64 v = src[(long)a * B + b];
      if (CONJ) v.y = -v.y;
      tile[k][tx] = v;
    }
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int b = b0 + k, a = a0 + tx;
    if (a < A && b < B) dst[(long)b * A + a] = tile[tx][k];
  }
}

__global__ void __launch_bounds__(NT)
k_transpose_real(const double* __restrict__ in, double* __restrict__ out, int A, int B) {
  __shared__ double tile[32][33];
  const int a0 = blockIdx.x * 32, b0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int a = a0 + k, b = b0 + tx;
    if (a < A && b < B) tile[k][tx] = in[(long)a * B + b];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int b = b0 + k, a = a0 + tx;
    if (a < A && b < B) out[(long)b * A + a] = tile[tx][k];
  }
}

inline int blocks_for(long n) {
  long b = (n + NT - 1) / NT;
  return (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}

}  // namespace

// ---------------------------------------------------------------- launchers
template <typename T>
void launch_proj(const cplx<T>* Phi, long ldphi, int nv, int npw, cplx<T>* Y, long ldy, const int* act,
                 int nsys, hipStream_t s) {
  if (nsys <= 0 || nv <= 0) return;
  k_proj<T><<<nsys, NT, 0, s>>>(Phi, ldphi, nv, npw, Y, ldy, act);
}

template <typename T>
void launch_cg_init(const SolveVecs<T>& v, const cplx<T>* b, long ldb, const int* bidx, int npw, int nsys,
                    bool keep_x, const int* act, hipStream_t s, const ProjFeed<T>& f, T* npart) {
  if (nsys <= 0) return;
  if (f.part)
    k_cg_init_fed<T><<<dim3(f.nsplit, nsys), NT, 0, s>>>(v, b, ldb, bidx, npw, keep_x ? 1 : 0, act, npart, f);
  else
    k_cg_init<T><<<nsys, NT, 0, s>>>(v, b, ldb, bidx, npw, keep_x ? 1 : 0, act);
}

template <typename T>
void launch_cg_step(const SolveVecs<T>& v, int npw, T tol2, const int* act, int nsys, hipStream_t s) {
  if (nsys <= 0) return;
  k_cg_step<T><<<nsys, NT, 0, s>>>(v, npw, tol2, act);
}

template <typename T>
void launch_sqmr_init(const SolveVecs<T>& v, const cplx<T>* b, long ldb, const int* bidx, int npw, int nsys,
                      bool keep_x, const int* act, hipStream_t s) {
  if (nsys <= 0) return;
  k_sqmr_init<T><<<nsys, NT, 0, s>>>(v, b, ldb, bidx, npw, keep_x ? 1 : 0, act);
}

template <typename T>
void launch_sqmr_step(const SolveVecs<T>& v, int npw, T tol, const int* act, int nsys, hipStream_t s) {
  if (nsys <= 0) return;
  k_sqmr_step<T><<<nsys, NT, 0, s>>>(v, npw, tol, act);
}

template <typename T>
void launch_resid(const cplx<T>* b, long ldb, const int* bidx, const cplx<T>* AX, long lda, cplx<T>* R,
                  long ldr, double* res, int npw, const int* act, int nsys, hipStream_t s) {
  if (nsys <= 0) return;
  k_resid<T><<<nsys, NT, 0, s>>>(b, ldb, bidx, AX, lda, R, ldr, res, npw, act);
}

template <typename T>
void launch_resid_split(const cplx<T>* b, long ldb, const int* bidx, const cplx<T>* AX, long lda, cplx<T>* R,
                        long ldr, double* res, int ns, int npw, const int* act, int nsys, hipStream_t s) {
  if (nsys <= 0) return;
  k_resid_split<T><<<dim3(ns, nsys), NT, 0, s>>>(b, ldb, bidx, AX, lda, R, ldr, res, npw, act);
}
template void launch_resid_split<double>(const z64*, long, const int*, const z64*, long, z64*, long, double*, int,
                                         int, const int*, int, hipStream_t);

void launch_dots(const z64* A, long lda, int m, const z64* w, long n, z64* h, z64* partial, hipStream_t s) {
  if (m <= 0) return;
  k_dots_partial<<<dim3(kDotBlocks, m), NT, 0, s>>>(A, lda, w, n, partial);
  k_dots_final<<<m, 64, 0, s>>>(partial, kDotBlocks, h);
}

void launch_cgs_pass(const z64* A, long lda, int m, z64* w, const z64* src, long n, z64* h, z64* partial,
                     double* re_last, hipStream_t s) {
  if (m <= 0) return;
  const z64* in = src ? src : w;
  k_dots_partial<<<dim3(kDotBlocks, m), NT, 0, s>>>(A, lda, in, n, partial);
  if (m <= kCgsMax) {
    k_cgs_sub<<<blocks_for(n), NT, 0, s>>>(A, lda, m, partial, kDotBlocks, w, src, n, re_last);
    return;
  }
  k_dots_final<<<m, 64, 0, s>>>(partial, kDotBlocks, h);
  if (re_last) k_re_of<<<1, 64, 0, s>>>(h + m - 1, re_last);
  if (src) k_copy<<<blocks_for(n), NT, 0, s>>>(src, w, n);
  k_gemv_sub<<<blocks_for(n), NT, 0, s>>>(A, lda, m, h, w, n);
}

void launch_gemv_sub(const z64* A, long lda, int m, const z64* h, z64* w, long n, hipStream_t s) {
  if (m <= 0) return;
  k_gemv_sub<<<blocks_for(n), NT, 0, s>>>(A, lda, m, h, w, n);
}

void launch_lanczos_alpha(const z64* q, const z64* w, long n, double* alpha_j, z64* partial, hipStream_t s) {
  k_dots_partial<<<dim3(kDotBlocks, 1), NT, 0, s>>>(q, 0, w, n, partial);
  k_alpha_final<<<1, 64, 0, s>>>(partial, kDotBlocks, alpha_j);
}

void launch_lanczos_sub(z64* w, const z64* q, const z64* qprev, const double* alpha_j, const double* beta_prev,
                        long n, hipStream_t s, const z64* src) {
  k_lanczos_sub<<<blocks_for(n), NT, 0, s>>>(w, q, qprev, alpha_j, beta_prev, n, src);
}

void launch_norm(const z64* w, long n, double* out, z64* partial, hipStream_t s, const double* alpha,
                 double* pair) {
  k_dots_partial<<<dim3(kDotBlocks, 1), NT, 0, s>>>(w, 0, w, n, partial);
  k_norm_final<<<1, 64, 0, s>>>(partial, kDotBlocks, out, alpha, pair);
}

void launch_scale_into(const z64* w, const double* nrm, z64* q, long n, hipStream_t s) {
  k_scale_into<<<blocks_for(n), NT, 0, s>>>(w, nrm, q, n);
}

void launch_axpby(z64* y, const z64* x, z64 a, z64 b, long n, hipStream_t s) {
  k_axpby<<<blocks_for(n), NT, 0, s>>>(y, x, a, b, n);
}

void launch_add(z64* y, const z64* a, const z64* b, long n, hipStream_t s) {
  k_add<<<blocks_for(n), NT, 0, s>>>(y, a, b, n);
}

void launch_finite_check(const double* x, long n, int* flag, hipStream_t s) {
  k_finite<<<blocks_for(n), NT, 0, s>>>(x, n, flag);
}

void launch_cvt_64_32(const z64* in, z32* out, long n, hipStream_t s) {
  k_cvt_64_32<<<blocks_for(n), NT, 0, s>>>(in, out, n);
}

void launch_cvt_32_64(const z32* in, z64* out, long n, hipStream_t s) {
  if (n <= 0) return;
  k_cvt_32_64<<<blocks_for(n), NT, 0, s>>>(in, out, n);
}

void launch_mul(z64* y, const z64* a, const z64* b, long n, hipStream_t s) {
  if (n <= 0) return;
  k_mul<<<blocks_for(n), NT, 0, s>>>(y, a, b, n);
}

template <class T>
void launch_fill(cplx<T>* p, cplx<T> v, long n, hipStream_t s) {
  if (n <= 0) return;
  k_fill<T><<<blocks_for(n), NT, 0, s>>>(p, v, n);
}
template void launch_fill<double>(z64*, z64, long, hipStream_t);
template void launch_fill<float>(z32*, z32, long, hipStream_t);

void launch_cvt_32_64_axpy(const z32* e, z64* x, const double* scale, const int* act, long ld, int npw,
                           int nsys, hipStream_t s, const float* d, bool assign) {
  if (nsys <= 0) return;
  k_cvt_32_64_axpy<<<dim3((npw + NT - 1) / NT, nsys), NT, 0, s>>>(e, x, scale, act, ld, npw, d, assign ? 1 : 0);
}

void launch_xyz_to_zxy(int N, const z64* in, long ldi, z64* out, long ldo, int nvec, bool conj_in,
                       hipStream_t s) {
  if (nvec <= 0) return;
  const int A = N * N, B = N;
  dim3 grid((A + 31) / 32, (B + 31) / 32, nvec);
  if (conj_in) k_transpose<true><<<grid, NT, 0, s>>>(in, ldi, out, ldo, A, B);
  else k_transpose<false><<<grid, NT, 0, s>>>(in, ldi, out, ldo, A, B);
}

void launch_zxy_to_xyz(int N, const z64* in, long ldi, z64* out, long ldo, int nvec, hipStream_t s) {
  if (nvec <= 0) return;
  const int A = N, B = N * N;
  dim3 grid((A + 31) / 32, (B + 31) / 32, nvec);
  k_transpose<false><<<grid, NT, 0, s>>>(in, ldi, out, ldo, A, B);
}

void launch_real_xyz_to_zxy(int N, const double* in, double* out, hipStream_t s) {
  const int A = N * N, B = N;
  dim3 grid((A + 31) / 32, (B + 31) / 32);
  k_transpose_real<<<grid, NT, 0, s>>>(in, out, A, B);
}

void launch_real_zxy_to_xyz(int N, const double* in, double* out, hipStream_t s) {
  const int A = N, B = N * N;
  dim3 grid((A + 31) / 32, (B + 31) / 32);
  k_transpose_real<<<grid, NT, 0, s>>>(in, out, A, B);
}

#define LGW_INST_S(T)                                                                                  \
  template void launch_proj<T>(const cplx<T>*, long, int, int, cplx<T>*, long, const int*, int,         \
                               hipStream_t);                                                           \
  template void launch_cg_init<T>(const SolveVecs<T>&, const cplx<T>*, long, const int*, int, int, bool,\
                                  const int*, hipStream_t, const ProjFeed<T>&, T*);                                \
  template void launch_cg_step<T>(const SolveVecs<T>&, int, T, const int*, int, hipStream_t);          \
  template void launch_sqmr_init<T>(const SolveVecs<T>&, const cplx<T>*, long, const int*, int, int,    \
                                    bool, const int*, hipStream_t);                                                \
  template void launch_sqmr_step<T>(const SolveVecs<T>&, int, T, const int*, int, hipStream_t);        \
  template void launch_resid<T>(const cplx<T>*, long, const int*, const cplx<T>*, long, cplx<T>*, long, \
                                double*, int, const int*, int, hipStream_t);

LGW_INST_S(double)
LGW_INST_S(float)

}  // namespace lgw

namespace lgw {
namespace {
// dst[didx[p]] = src[a[p]] (+ src[b[p]])
__global__ void __launch_bounds__(256)
k_rows_out(const z64* __restrict__ src, long lds, z64* __restrict__ dst, long ldd,
           const int* __restrict__ didx, const int* __restrict__ a, const int* __restrict__ b, int n) {
  const int p = blockIdx.y;
  const z64* sa = src + (long)a[p] * lds;
  const z64* sb = b ? src + (long)b[p] * lds : nullptr;
  z64* d = dst + (long)didx[p] * ldd;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    z64 v = sa[i];
    if (sb) v = v + sb[i];
    d[i] = v;
  }
}

// out32[sys] = in64[sys] * inv[sys]
__global__ void __launch_bounds__(256)
k_scale_cvt(const z64* __restrict__ in, long ldi, z32* __restrict__ out, long ldo,
            const double* __restrict__ scale, const int* __restrict__ act, int n, const float* __restrict__ d) {
  const int sys = sys_of(act, blockIdx.y);
  const double s = scale[sys];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const z32 v = cvt<float>(s * in[(long)sys * ldi + i]);
    out[(long)sys * ldo + i] = d ? d[i] * v : v;
  }
}

// Y[yrow] = d * X[xrow] elementwise over the first n entries, row i of the
// grid taking xrow = xi ? xi[i] : i and yrow = yi ? yi[i] : i (X == Y allowed)
template <typename T>
__global__ void __launch_bounds__(256)
k_scale_diag(const cplx<T>* X, long ldx, const int* __restrict__ xi, cplx<T>* Y, long ldy,
             const int* __restrict__ yi, const T* __restrict__ d, int n) {
  const int xr = xi ? xi[blockIdx.y] : (int)blockIdx.y;
  const int yr = yi ? yi[blockIdx.y] : (int)blockIdx.y;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
    Y[(long)yr * ldy + i] = d[i] * X[(long)xr * ldx + i];
}

// sum_b conj(A[a]) B[b] over n for a < m, b < p: C[b][a]; one workgroup per (a-tile, b)
__global__ void __launch_bounds__(256)
k_gemm_hn_partial(const z64* __restrict__ A, long lda, int m, const z64* __restrict__ B, long ldb,
                  long n, int nsplit, z64* __restrict__ partial) {
  // grid: (nsplit, p); each workgroup handles one B row and all m A rows over a slice of n
  __shared__ double sm[2 * 8 * 4];
  const int bcol = blockIdx.y;
  const long chunk = (n + nsplit - 1) / nsplit;
  const long e0 = (long)blockIdx.x * chunk;
  const long e1 = e0 + chunk < n ? e0 + chunk : n;
  const z64* bb = B + (long)bcol * ldb;
  for (int a0 = 0; a0 < m; a0 += 8) {
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    for (long e = e0 + threadIdx.x; e < e1; e += 256) {
      const z64 bv = bb[e];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (a0 + u < m) {
          const z64 p = cmulc(A[(long)(a0 + u) * lda + e], bv);
          acc[2 * u] += p.x;
          acc[2 * u + 1] += p.y;
        }
      }
    }
    // block reduce 16 values
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      double s = acc[u];
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
      if (lane == 0) sm[u * 4 + w] = s;
    }
    __syncthreads();
    if (threadIdx.x < 8 && a0 + (int)threadIdx.x < m) {
      const int u = threadIdx.x;
      const double re = sm[(2 * u) * 4 + 0] + sm[(2 * u) * 4 + 1] + sm[(2 * u) * 4 + 2] + sm[(2 * u) * 4 + 3];
      const double im = sm[(2 * u + 1) * 4 + 0] + sm[(2 * u + 1) * 4 + 1] + sm[(2 * u + 1) * 4 + 2] +
                        sm[(2 * u + 1) * 4 + 3];
      partial[((long)bcol * m + a0 + u) * nsplit + blockIdx.x] = z64{re, im};
    }
    __syncthreads();
  }
}

__global__ void k_gemm_hn_final(const z64* __restrict__ partial, int nsplit, z64* __restrict__ C, int total) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < total) {
    z64 s{0, 0};
    for (int k = 0; k < nsplit; ++k) s = s + partial[(long)i * nsplit + k];
    C[i] = s;
  }
}
}  // namespace

void launch_rows_out(const z64* src, long lds, z64* dst, long ldd, const int* didx, const int* a, const int* b,
                     int n, int np, hipStream_t s) {
  if (np <= 0) return;
  k_rows_out<<<dim3((n + 255) / 256, np), 256, 0, s>>>(src, lds, dst, ldd, didx, a, b, n);
}

void launch_scale_cvt(const z64* in, long ldi, z32* out, long ldo, const double* scale, const int* act, int n,
                      int nsys, hipStream_t s, const float* d) {
  if (nsys <= 0) return;
  k_scale_cvt<<<dim3((n + 255) / 256, nsys), 256, 0, s>>>(in, ldi, out, ldo, scale, act, n, d);
}

template <typename T>
void launch_scale_diag(const cplx<T>* X, long ldx, const int* xi, cplx<T>* Y, long ldy, const int* yi, const T* d,
                       int n, int nrows, hipStream_t s) {
  if (nrows <= 0 || n <= 0) return;
  k_scale_diag<T><<<dim3((n + 255) / 256, nrows), 256, 0, s>>>(X, ldx, xi, Y, ldy, yi, d, n);
}
template void launch_scale_diag<double>(const z64*, long, const int*, z64*, long, const int*, const double*, int,
                                        int, hipStream_t);
template void launch_scale_diag<float>(const z32*, long, const int*, z32*, long, const int*, const float*, int, int,
                                       hipStream_t);

// C[b][a] = sum_e conj(A[a][e]) B[b][e], a < m, b < p; partial needs m*p*64 entries
void launch_gemm_hn(const z64* A, long lda, int m, const z64* B, long ldb, int p, long n, z64* C, z64* partial,
                    hipStream_t s) {
  if (m <= 0 || p <= 0) return;
  const int nsplit = 64;
  k_gemm_hn_partial<<<dim3(nsplit, p), 256, 0, s>>>(A, lda, m, B, ldb, n, nsplit, partial);
  k_gemm_hn_final<<<(m * p + 255) / 256, 256, 0, s>>>(partial, nsplit, C, m * p);
}
}  // namespace lgw

// ====================================================================
// Projector on the matrix cores.  C = Phi^H Y (bands x systems) reduces over
// the plane-wave index, a GEMM with a long K: one wave computes a 16 x 16
// MFMA tile whose rows are the real and imaginary parts of 8 bands and whose
// columns are 16 systems, over a slice of K; partial tiles are summed by the
// update kernel, which then applies Y -= Phi C streaming Y once.
namespace lgw {
namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16], B[l/16][l%16] and
// D[4j + l/16][l%16], j = 0..3.  Row r = 4j + q carries band q + 4(j/2),
// real part for even j, imaginary part for odd j.
template <> struct Mfma<double> {
  using acc = d4v;
  __device__ static acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static void row_role(int r, int& band, int& part) {
    const int q = r & 3, j = r >> 2;
    band = q + 4 * (j >> 1);
    part = j & 1;
  }
  // band of accumulator pair (re-reg jr, im-reg ji) for lane l: pairs (0,1), (2,3)
  __device__ static int out_band(int lane, int pair) { return (lane >> 4) + 4 * pair; }
};
// v_mfma_f32_16x16x4f32: D[4(l/16) + j][l%16].  Row r = 4q + j carries band
// 2q + j/2, real part for even j, imaginary for odd j.
template <> struct Mfma<float> {
  using acc = f4v;
  __device__ static acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static void row_role(int r, int& band, int& part) {
    const int q = r >> 2, j = r & 3;
    band = 2 * q + (j >> 1);
    part = j & 1;
  }
  __device__ static int out_band(int lane, int pair) { return 2 * (lane >> 4) + pair; }
};

constexpr int kProjGroups = kMaxBands / 8;

// grid (ks, ceil(nsys/16)), one wave: partial[ks][sys][v] = sum over the
// slice of conj(Phi_v) (d .* Y_sys), d = dpre or 1
template <typename T, int NG>
__global__ void __launch_bounds__(64)
k_proj_dots(const cplx<T>* __restrict__ Phi, long ldphi, int nv, int npw, const cplx<T>* __restrict__ Y,
            long ldy, const int* __restrict__ act, int nsys, int kchunk, cplx<T>* __restrict__ part,
            const T* __restrict__ dpre) {
  using M = Mfma<T>;
  const int lane = threadIdx.x;
  const int tile = blockIdx.y * 16;
  const int col = lane & 15, kl = lane >> 4;
  const int sidx = tile + col;
  const bool svalid = sidx < nsys;
  const int sys = svalid ? sys_of(act, sidx) : 0;
  const cplx<T>* Ys = Y + (long)sys * ldy;
  const int r = lane & 15;
  int band, partv;
  M::row_role(r, band, partv);
  constexpr int ngroups = NG;
  typename M::acc c1[NG], c2[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    c1[g] = typename M::acc{0, 0, 0, 0};
    c2[g] = typename M::acc{0, 0, 0, 0};
  }
  const int k_begin = blockIdx.x * kchunk;
  const int k_end = min(npw, k_begin + kchunk);
  constexpr int U = 4;   // K steps of 4 loaded ahead of their MFMAs
  for (int k0 = k_begin; k0 < k_end; k0 += 4 * U) {
    cplx<T> y[U];
    T a[U][NG];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kk = k0 + 4 * u + kl;
      const bool kv = kk < k_end;
      y[u] = (kv && svalid) ? Ys[kk] : cplx<T>{0, 0};
      if (dpre && kv) y[u] = dpre[kk] * y[u];
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        a[u][g] = T(0);
        const int v = 8 * g + band;
        if (g < ngroups && kv && v < nv) {
          const cplx<T> p = Phi[(long)v * ldphi + kk];
          a[u][g] = partv ? p.y : p.x;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        if (g < ngroups) {
          c1[g] = M::mma(a[u][g], y[u].x, c1[g]);
          c2[g] = M::mma(a[u][g], y[u].y, c2[g]);
        }
      }
    }
  }
  if (!svalid) return;
  cplx<T>* P = part + ((long)blockIdx.x * nsys + sidx) * nv;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    if (g < ngroups) {
#pragma unroll
      for (int pr = 0; pr < 2; ++pr) {
        const int v = 8 * g + M::out_band(lane, pr);
        const int jr = 2 * pr, ji = 2 * pr + 1;
        if (v < nv) P[v] = cplx<T>{c1[g][jr] + c2[g][ji], c2[g][jr] - c1[g][ji]};
      }
    }
  }
}

// grid (ceil(npw/256), ceil(nsys/16)):
//   Y_sys = dpost .* (dpre .* X_sys - sum_v Phi_v C[v][sys])   (X may be Y)
template <typename T>
__global__ void __launch_bounds__(256)
k_proj_update(const cplx<T>* __restrict__ Phi, long ldphi, int nv, int npw, const cplx<T>* X, cplx<T>* Y,
              long ldy, const int* __restrict__ act, int nsys, int ks, const cplx<T>* __restrict__ part,
              const T* __restrict__ dpre, const T* __restrict__ dpost) {
  __shared__ cplx<T> C[16][kMaxBands];
  __shared__ cplx<T> red[256];
  const int tile = blockIdx.y * 16;
  const int nt = min(16, nsys - tile);
  // C = sum of the ks partial tiles: tpe threads per entry (a power of two,
  // at least 16 so a long K-split is summed in parallel), rounds of 256/tpe
  // entries, fixed order (strided partial sums, then a tree in LDS)
  const int E = nt * nv;
  constexpr int tpe = 16;
  constexpr int per_round = 256 / tpe;
  const int sub = threadIdx.x % tpe;
  for (int e0 = 0; e0 < E; e0 += per_round) {
    const int e = e0 + threadIdx.x / tpe;
    cplx<T> a0{0, 0}, a1{0, 0};
    if (e < E) {
      const int s = e / nv, v = e - s * nv;
      const cplx<T>* pp = part + (long)(tile + s) * nv + v;
      const long step = (long)nsys * nv;
      int k = sub;
      for (; k + tpe < ks; k += 2 * tpe) {
        a0 = a0 + pp[(long)k * step];
        a1 = a1 + pp[(long)(k + tpe) * step];
      }
      if (k < ks) a0 = a0 + pp[(long)k * step];
    }
    red[threadIdx.x] = a0 + a1;
    __syncthreads();
#pragma unroll
    for (int off = tpe / 2; off > 0; off >>= 1) {
      if (sub < off) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + off];
      __syncthreads();
    }
    if (sub == 0 && e < E) {
      const int s = e / nv, v = e - s * nv;
      C[s][v] = red[threadIdx.x];
    }
    __syncthreads();
  }
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= npw) return;
  for (int v0 = 0; v0 < nv; v0 += 8) {
    cplx<T> ph[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) ph[u] = v0 + u < nv ? Phi[(long)(v0 + u) * ldphi + i] : cplx<T>{0, 0};
    for (int s0 = 0; s0 < nt; s0 += 4) {
      cplx<T> y[4];
      long row[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        row[q] = s0 + q < nt ? (long)sys_of(act, tile + s0 + q) * ldy : -1;
        y[q] = row[q] >= 0 ? (v0 == 0 ? X[row[q] + i] : Y[row[q] + i]) : cplx<T>{0, 0};
        if (v0 == 0 && dpre) y[q] = dpre[i] * y[q];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (row[q] < 0) continue;
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (v0 + u < nv) y[q] = y[q] - C[s0 + q][v0 + u] * ph[u];
        if (dpost && v0 + 8 >= nv) y[q] = dpost[i] * y[q];
        Y[row[q] + i] = y[q];
      }
    }
  }
}

}  // namespace

// total single-wave workgroups the projector's dots launch aims for
#ifndef LGW_PROJ_WAVES
#define LGW_PROJ_WAVES 2048
#endif

template <typename T>
int proj_ksplit(int npw, int nsys) {
  const int tiles = (nsys + 15) / 16;
  int ks = (LGW_PROJ_WAVES + tiles - 1) / tiles;
  const int kmax = (npw + 63) / 64;         // keep slices >= 64 plane waves
  if (ks > kmax) ks = kmax;
  return ks < 1 ? 1 : ks;
}

template <typename T>
void launch_proj_mfma(const cplx<T>* Phi, long ldphi, int nv, int npw, const cplx<T>* X, cplx<T>* Y, long ldy,
                      const int* act, int nsys, cplx<T>* part, const T* dpre, const T* dpost, hipStream_t s) {
  if (nsys <= 0 || nv <= 0) return;
  const int ks = proj_ksplit<T>(npw, nsys);
  int kchunk = (npw + ks - 1) / ks;
  kchunk = (kchunk + 3) & ~3;
  const int tiles = (nsys + 15) / 16;
  const dim3 grid(ks, tiles);
  switch ((nv + 7) / 8) {
    case 1: k_proj_dots<T, 1><<<grid, 64, 0, s>>>(Phi, ldphi, nv, npw, X, ldy, act, nsys, kchunk, part, dpre); break;
    case 2: k_proj_dots<T, 2><<<grid, 64, 0, s>>>(Phi, ldphi, nv, npw, X, ldy, act, nsys, kchunk, part, dpre); break;
    case 3: k_proj_dots<T, 3><<<grid, 64, 0, s>>>(Phi, ldphi, nv, npw, X, ldy, act, nsys, kchunk, part, dpre); break;
    default: k_proj_dots<T, 4><<<grid, 64, 0, s>>>(Phi, ldphi, nv, npw, X, ldy, act, nsys, kchunk, part, dpre); break;
  }
  k_proj_update<T><<<dim3((npw + 255) / 256, tiles), 256, 0, s>>>(Phi, ldphi, nv, npw, X, Y, ldy, act, nsys, ks,
                                                                   part, dpre, dpost);
}


template <typename T>
void launch_proj_mfma(const cplx<T>* Phi, long ldphi, int nv, int npw, cplx<T>* Y, long ldy, const int* act,
                      int nsys, cplx<T>* part, hipStream_t s) {
  launch_proj_mfma<T>(Phi, ldphi, nv, npw, Y, Y, ldy, act, nsys, part, nullptr, nullptr, s);
}

// C[b * ldc + a] = sum over the ks slices of part[k][b][a] (a < mb), in slice order
__global__ void __launch_bounds__(256) k_sum_slices(const z64* __restrict__ part, int ks, int p, int mb,
                                                    z64* __restrict__ C, long ldc) {
  const long total = (long)p * mb;
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  z64 acc{0, 0};
  for (int k = 0; k < ks; ++k) acc = acc + part[(long)k * total + i];
  const long b = i / mb;
  C[b * ldc + (i - b * mb)] = acc;
}

// C^T block of C[b][a] = sum_e conj(A[a][e]) B[b][e]: one workgroup takes a
// K range and 128 rows of B against up to 64 rows of A.  Chunks of 16 K
// elements of both are staged in LDS with row-contiguous loads; each wave then
// computes a 64 x 32 block (four 16-row A tiles by two 16-row B tiles) on
// v_mfma_f64_16x16x4f64 (lane l: A[l%16][l/16], B[l/16][l%16],
// D[4r + l/16][l%16]), the complex product as four real ones, and writes
// partial[slice][b][a].
constexpr int kGemmKC = 16;                // K elements per LDS chunk
constexpr int kGemmBRows = 128;            // B rows per workgroup
constexpr int kGemmLd = kGemmKC + 1;       // padded LDS row (complex values)
__global__ void __launch_bounds__(256)
k_gemm_hn_tiled(const z64* __restrict__ A, long lda, int mb, const z64* __restrict__ B, long ldb, int p, long n,
                long kchunk, z64* __restrict__ partial) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  __shared__ z64 As[64 * kGemmLd];
  __shared__ z64 Bs[kGemmBRows * kGemmLd];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = lane & 15, kl = lane >> 4;
  const int b0 = blockIdx.y * kGemmBRows;
  const long e_begin = (long)blockIdx.x * kchunk;
  const long e_end = e_begin + kchunk < n ? e_begin + kchunk : n;
  d4 cr[4][2], ci[4][2];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      cr[m][q] = d4{0, 0, 0, 0};
      ci[m][q] = d4{0, 0, 0, 0};
    }
  const int lr = threadIdx.x >> 4, le = threadIdx.x & 15;   // loader: 16 rows x 16 elements per pass
  for (long e0 = e_begin; e0 < e_end; e0 += kGemmKC) {
    const long e = e0 + le;
    const bool ev = e < e_end;
#pragma unroll
    for (int r = lr; r < 64; r += 16) As[r * kGemmLd + le] = (ev && r < mb) ? A[(long)r * lda + e] : z64{0, 0};
#pragma unroll
    for (int r = lr; r < kGemmBRows; r += 16)
      Bs[r * kGemmLd + le] = (ev && b0 + r < p) ? B[(long)(b0 + r) * ldb + e] : z64{0, 0};
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < kGemmKC; k4 += 4) {
      z64 av[4], bv[2];
#pragma unroll
      for (int m = 0; m < 4; ++m) av[m] = As[(16 * m + col) * kGemmLd + k4 + kl];
#pragma unroll
      for (int q = 0; q < 2; ++q) bv[q] = Bs[(32 * w + 16 * q + col) * kGemmLd + k4 + kl];
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          // conj(a) b = (ar br + ai bi) + i (ar bi - ai br)
          cr[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[m].x, bv[q].x, cr[m][q], 0, 0, 0);
          cr[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[m].y, bv[q].y, cr[m][q], 0, 0, 0);
          ci[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[m].x, bv[q].y, ci[m][q], 0, 0, 0);
          ci[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[m].y, bv[q].x, ci[m][q], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  z64* P = partial + (long)blockIdx.x * p * mb;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * m + 4 * r + kl;
        const int b = b0 + 32 * w + 16 * q + col;
        if (a < mb && b < p) P[(long)b * mb + a] = z64{cr[m][q][r], ci[m][q][r]};
      }
}

int gemm_hn_slices(long n, int p) {
  const int btiles = (p + kGemmBRows - 1) / kGemmBRows;
  int ks = (1024 + btiles - 1) / btiles;                  // about four workgroups per compute unit
  const long kmax = (n + 8 * kGemmKC - 1) / (8 * kGemmKC);   // at least 8 chunks per slice
  if (ks > kmax) ks = (int)kmax;
  return ks < 1 ? 1 : ks;
}

// Blocks of up to 64 rows of A: partial[k][b][a] from the tiled kernel, then
// the slice sum into C's columns of the block.
void launch_gemm_hn_mfma(const z64* A, long lda, int m, const z64* B, long ldb, int p, long n, z64* C, z64* partial,
                         hipStream_t s) {
  if (m <= 0 || p <= 0 || n <= 0) return;
  const int ks = gemm_hn_slices(n, p);
  long kchunk = (n + ks - 1) / ks;
  kchunk = (kchunk + kGemmKC - 1) / kGemmKC * kGemmKC;
  const dim3 grid(ks, (p + kGemmBRows - 1) / kGemmBRows);
  for (int a0 = 0; a0 < m; a0 += 64) {
    const int mb = m - a0 < 64 ? m - a0 : 64;
    k_gemm_hn_tiled<<<grid, 256, 0, s>>>(A + (long)a0 * lda, lda, mb, B, ldb, p, n, kchunk, partial);
    const long total = (long)p * mb;
    k_sum_slices<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(partial, ks, p, mb, C + a0, m);
  }
}

template int proj_ksplit<double>(int, int);
template int proj_ksplit<float>(int, int);
template void launch_proj_mfma<double>(const z64*, long, int, int, z64*, long, const int*, int, z64*, hipStream_t);
template void launch_proj_mfma<float>(const z32*, long, int, int, z32*, long, const int*, int, z32*, hipStream_t);
template void launch_proj_mfma<double>(const z64*, long, int, int, const z64*, z64*, long, const int*, int, z64*,
                                       const double*, const double*, hipStream_t);
template void launch_proj_mfma<float>(const z32*, long, int, int, const z32*, z32*, long, const int*, int, z32*,
                                      const float*, const float*, hipStream_t);

}  // namespace lgw

namespace lgw {
namespace {
// W[c] -= sum_{i<m} X[i] Cm[c][i] for c < b (grid vectors of length n)
__global__ void __launch_bounds__(256)
k_block_sub(z64* __restrict__ W, long ldw, int b, const z64* __restrict__ X, long ldx, int m,
            const z64* __restrict__ Cm, long n) {
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    for (int c = 0; c < b; ++c) {
      z64 acc = W[(long)c * ldw + e];
      const z64* cc = Cm + (long)c * m;
      for (int i = 0; i < m; ++i) acc = acc - cc[i] * X[(long)i * ldx + e];
      W[(long)c * ldw + e] = acc;
    }
  }
}
}  // namespace

void launch_block_sub(z64* W, long ldw, int b, const z64* X, long ldx, int m, const z64* Cm, long n,
                      hipStream_t s) {
  if (b <= 0 || m <= 0) return;
  long blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  k_block_sub<<<(int)blocks, 256, 0, s>>>(W, ldw, b, X, ldx, m, Cm, n);
}
}  // namespace lgw

namespace lgw {
namespace {
// out[e] += Re(c * conj(a[e]) * b[e])  (grid accumulation of the adjoint terms)
__global__ void __launch_bounds__(256)
k_acc_re(double* __restrict__ out, const z64* __restrict__ a, const z64* __restrict__ b, z64 c, long n) {
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) {
    const z64 p = c * cmulc(a[e], b[e]);
    out[e] += p.x;
  }
}
__global__ void __launch_bounds__(256)
k_conj(const z64* __restrict__ in, z64* __restrict__ out, long n) {
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long)gridDim.x * 256) out[e] = conj(in[e]);
}
}  // namespace

void launch_acc_re(double* out, const z64* a, const z64* b, z64 c, long n, hipStream_t s) {
  long blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  k_acc_re<<<(int)blocks, 256, 0, s>>>(out, a, b, c, n);
}
void launch_conj(const z64* in, z64* out, long n, hipStream_t s) {
  long blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  k_conj<<<(int)blocks, 256, 0, s>>>(in, out, n);
}
}  // namespace lgw

// ====================================================================
// Split Krylov updates for small batches: a system's vectors are spread over
// `nsplit` workgroups, with the block reductions exchanged through a small
// partial-sum buffer between three kernels (dots; x/r update + new norm;
// search-direction update).  Every workgroup rebuilds the same scalars from
// the partials in a fixed order, so the result matches the one-workgroup
// kernels up to the summation order.
namespace lgw {
namespace {

template <typename T>
__device__ __forceinline__ void slice_of(int npw, int nsplit, int& i0, int& i1) {
  const int chunk = (npw + nsplit - 1) / nsplit;
  i0 = blockIdx.x * chunk;
  i1 = min(npw, i0 + chunk);
}

// Partials are indexed by active slot (blockIdx.y), not by system.
// phase 1: part[slot][blk] = Re p^H Ap.  Workgroup 0 first commits the norm
// the previous phase 3 parked in theta (rr itself is never written while a
// launch may still read it).
template <typename T>
__global__ void __launch_bounds__(NT)
k_cg_split1(SolveVecs<T> v, int npw, const int* __restrict__ act, int nsplit, T* __restrict__ part) {
  __shared__ T sm[NT / 64];
  const int sys = sys_of(act, blockIdx.y);
  if (v.flag[sys]) return;
  if (blockIdx.x == 0 && threadIdx.x == 0 && v.theta[sys] >= T(0)) {
    v.rr[sys] = v.theta[sys];
    v.theta[sys] = T(-1);
  }
  int i0, i1;
  slice_of<T>(npw, nsplit, i0, i1);
  const cplx<T>* p = v.p + (long)sys * v.ld;
  const cplx<T>* Ap = v.Ap + (long)sys * v.ld;
  T acc[1] = {T(0)};
  for (int i = i0 + threadIdx.x; i < i1; i += NT) acc[0] += p[i].x * Ap[i].x + p[i].y * Ap[i].y;
  block_sum<T, 1>(acc, sm);
  if (threadIdx.x == 0) part[(long)blockIdx.y * nsplit + blockIdx.x] = acc[0];
}

// phase 2: alpha from the partials; x += alpha p; r -= alpha Ap; |r|^2 partials
template <typename T>
__global__ void __launch_bounds__(NT)
k_cg_split2(SolveVecs<T> v, int npw, const int* __restrict__ act, int nsplit, const T* __restrict__ part,
            T* __restrict__ part2) {
  __shared__ T sm[NT / 64];
  const int sys = sys_of(act, blockIdx.y);
  if (v.flag[sys]) return;
  T pAp = T(0);
  for (int k = 0; k < nsplit; ++k) pAp += part[(long)blockIdx.y * nsplit + k];
  if (!(pAp > T(0))) {
    if (blockIdx.x == 0 && threadIdx.x == 0) v.flag[sys] = FLAG_BREAK;
    return;
  }
  const T alpha = v.rr[sys] / pAp;
  int i0, i1;
  slice_of<T>(npw, nsplit, i0, i1);
  cplx<T>* x = v.x + (long)sys * v.ld;
  cplx<T>* r = v.r + (long)sys * v.ld;
  const cplx<T>* p = v.p + (long)sys * v.ld;
  const cplx<T>* Ap = v.Ap + (long)sys * v.ld;
  T acc[1] = {T(0)};
  for (int i = i0 + threadIdx.x; i < i1; i += NT) {
    x[i] = x[i] + alpha * p[i];
    const cplx<T> ri = r[i] - alpha * Ap[i];
    r[i] = ri;
    acc[0] += norm2(ri);
  }
  block_sum<T, 1>(acc, sm);
  if (threadIdx.x == 0) part2[(long)blockIdx.y * nsplit + blockIdx.x] = acc[0];
}

// phase 3: beta from the partials; p = r + beta p; workgroup 0 parks the new
// norm in theta and updates the iteration count and the convergence flag
template <typename T>
__global__ void __launch_bounds__(NT)
k_cg_split3(SolveVecs<T> v, int npw, T tol2, const int* __restrict__ act, int nsplit, const T* __restrict__ part2) {
  const int sys = sys_of(act, blockIdx.y);
  if (v.flag[sys]) return;
  T rrn = T(0);
  for (int k = 0; k < nsplit; ++k) rrn += part2[(long)blockIdx.y * nsplit + k];
  const T beta = rrn / v.rr[sys];
  int i0, i1;
  slice_of<T>(npw, nsplit, i0, i1);
  cplx<T>* p = v.p + (long)sys * v.ld;
  const cplx<T>* r = v.r + (long)sys * v.ld;
  for (int i = i0 + threadIdx.x; i < i1; i += NT) p[i] = r[i] + beta * p[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    v.theta[sys] = rrn;
    v.iters[sys] += 1;
    if (rrn <= tol2 * v.bb[sys]) v.flag[sys] = FLAG_CONV;
  }
}

// The x/r phase of a small preconditioned CG batch's step whose direction
// update and p^H A p are done by the transforms (launch_cg_step_fed).  The slice sums of
// conj(Phi_v) (pre .* r_new) are left for the next projection; the norm goes
// through a ticket: each workgroup stores its slice norm, the last of the
// system to take a ticket (all have read rr and the flag by then) sums them
// in a fixed order, parks the norm in theta, counts the step, sets the flag
// and returns the counter to zero.
template <typename T>
__global__ void __launch_bounds__(NT)
k_cg_split2f(SolveVecs<T> v, int npw, T tol2, const int* __restrict__ act, int nsplit, const T* __restrict__ dots,
             int ndots, T* __restrict__ part2, ProjFeed<T> f) {
  // points per thread whose loads are issued together (a slice of about 1024
  // points over 256 threads); partial sums of p^H A p loaded side by side
  constexpr int KB = sizeof(T) == 4 ? 5 : 2;
  constexpr int KD = sizeof(T) == 4 ? 32 : 16;
  __shared__ T sm[16 * (NT / 64)];
  const int slot = blockIdx.y;
  const int sys = sys_of(act, slot);
  int i0, i1;
  slice_of<T>(npw, nsplit, i0, i1);
  const long off = (long)sys * v.ld;
  cplx<T>* x = v.x + off;
  cplx<T>* r = v.r + off;
  const cplx<T>* p = v.p + off;
  const cplx<T>* Ap = v.Ap + off;
  // Every load that depends only on the system is issued before the flag,
  // alpha and the stores are decided: the memory latency is paid about once
  // instead of once per dependent step (a point's stores would otherwise
  // hold back the next point's loads).  Slots past the slice read its first
  // point (point 0 for an empty slice) and drop it.
  const int base = i0 < i1 ? i0 : 0;
  const int flag = v.flag[sys];
  const T rr = v.rr[sys];
  T dv[KD];
#pragma unroll
  for (int k = 0; k < KD; ++k) dv[k] = dots[(long)slot * ndots + (k < ndots ? k : 0)];
  cplx<T> pv[KB], av[KB], rv[KB], xv[KB], ph[KB][8];
  T scv[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int i = i0 + threadIdx.x + k * NT;
    const int is = i < i1 ? i : base;
    pv[k] = p[is];
    av[k] = Ap[is];
    rv[k] = r[is];
    xv[k] = x[is];
    scv[k] = f.pre ? f.pre[is] : T(1);
#pragma unroll
    for (int u = 0; u < 8; ++u) ph[k][u] = u < f.nv ? f.Phi[(long)u * f.ldphi + is] : cplx<T>{0, 0};
  }
  if (flag) return;
  T pAp = T(0);
#pragma unroll
  for (int k = 0; k < KD; ++k)
    if (k < ndots) pAp += dv[k];
  for (int k = KD; k < ndots; ++k) pAp += dots[(long)slot * ndots + k];
  if (!(pAp > T(0))) {
    if (blockIdx.x == 0 && threadIdx.x == 0) v.flag[sys] = FLAG_BREAK;
    return;
  }
  const T alpha = rr / pAp;
  T acc[1] = {T(0)};
  T fa[16];
  feed_zero(fa);
  auto step = [&](int i, cplx<T> pi, cplx<T> ai, cplx<T> ri, cplx<T> xi, T sc, const cplx<T> (&phi)[8]) {
    x[i] = xi + alpha * pi;
    const cplx<T> rn = ri - alpha * ai;
    r[i] = rn;
    acc[0] += norm2(rn);
    const cplx<T> y = sc * rn;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      fa[2 * u] += phi[u].x * y.x + phi[u].y * y.y;
      fa[2 * u + 1] += phi[u].x * y.y - phi[u].y * y.x;
    }
  };
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int i = i0 + threadIdx.x + k * NT;
    if (i < i1) step(i, pv[k], av[k], rv[k], xv[k], scv[k], ph[k]);
  }
  for (int i = i0 + threadIdx.x + KB * NT; i < i1; i += NT) {
    // every load of the point before its stores
    const cplx<T> pi = p[i], ai = Ap[i], ri = r[i], xi = x[i];
    cplx<T> phi[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) phi[u] = u < f.nv ? f.Phi[(long)u * f.ldphi + i] : cplx<T>{0, 0};
    step(i, pi, ai, ri, xi, f.pre ? f.pre[i] : T(1), phi);
  }
  block_sum<T, 1>(acc, sm);
  feed_store(f, 0, blockIdx.x, sys, fa, sm);
  for (int v0 = 8; v0 < f.nv; v0 += 8) {
    feed_zero(fa);
    for (int i = i0 + threadIdx.x; i < i1; i += NT) feed_acc(f, v0, i, r[i], fa);
    feed_store(f, v0, blockIdx.x, sys, fa, sm);
  }
  __shared__ int last;
  if (threadIdx.x == 0) {
    part2[(long)slot * nsplit + blockIdx.x] = acc[0];
    const int ticket = __hip_atomic_fetch_add(v.cnt + slot, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = ticket == nsplit - 1;
  }
  __syncthreads();
  if (!last || threadIdx.x >= 64) return;
  // the last workgroup's first wave: the slice norms loaded side by side, then
  // a fixed shuffle tree (nsplit <= 64)
  T e = threadIdx.x < nsplit
            ? __hip_atomic_load(part2 + (long)slot * nsplit + threadIdx.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
            : T(0);
  const T rrn = wave_sum(e);
  if (threadIdx.x != 0) return;
  v.cnt[slot] = 0;
  v.theta[sys] = rrn;
  v.iters[sys] += 1;
  if (rrn <= tol2 * v.bb[sys]) v.flag[sys] = FLAG_CONV;
}

}  // namespace

template <typename T>
void launch_cg_step_split(const SolveVecs<T>& v, int npw, T tol2, const int* act, int nsys, int nsplit, T* part,
                          hipStream_t s) {
  if (nsys <= 0) return;
  const dim3 grid(nsplit, nsys);
  k_cg_split1<T><<<grid, NT, 0, s>>>(v, npw, act, nsplit, part);
  k_cg_split2<T><<<grid, NT, 0, s>>>(v, npw, act, nsplit, part, part + (long)nsys * nsplit);
  k_cg_split3<T><<<grid, NT, 0, s>>>(v, npw, tol2, act, nsplit, part + (long)nsys * nsplit);
}

template <typename T>
void launch_cg_step_fed(const SolveVecs<T>& v, int npw, T tol2, const int* act, int nsys, int nsplit, T* part,
                        const T* dots, int ndots, const ProjFeed<T>& f, hipStream_t s) {
  if (nsys <= 0) return;
  k_cg_split2f<T><<<dim3(nsplit, nsys), NT, 0, s>>>(v, npw, tol2, act, nsplit, dots, ndots, part, f);
}
template void launch_cg_step_fed<double>(const SolveVecs<double>&, int, double, const int*, int, int, double*,
                                         const double*, int, const ProjFeed<double>&, hipStream_t);
template void launch_cg_step_fed<float>(const SolveVecs<float>&, int, float, const int*, int, int, float*,
                                        const float*, int, const ProjFeed<float>&, hipStream_t);

template void launch_cg_step_split<double>(const SolveVecs<double>&, int, double, const int*, int, int, double*,
                                           hipStream_t);
template void launch_cg_step_split<float>(const SolveVecs<float>&, int, float, const int*, int, int, float*,
                                          hipStream_t);
}  // namespace lgw

// ====================================================================
// Multi-shift solves: one plain Lanczos recursion per system on
// A = P (H - e) P from its right-hand side serves every shift (the Krylov
// space of A - tau is that of A); see multishift() in the library.
namespace lgw {
namespace {
// Q[s][0] = b_s / |b_s|, nrm[s] = |b_s|; b_s = B[bidx[s]]
__global__ void __launch_bounds__(NT)
k_ms_init(const z64* __restrict__ B, long ldb, const int* __restrict__ bidx, int npw, z64* __restrict__ Q,
          long ldq, double* __restrict__ nrm) {
  __shared__ double sm[NT / 64];
  const int s = blockIdx.x;
  const z64* b = B + (long)bidx[s] * ldb;
  double acc[1] = {0.0};
  for (int i = threadIdx.x; i < npw; i += NT) acc[0] += norm2(b[i]);
  block_sum<double, 1>(acc, sm);
  const double n = sqrt(acc[0]);
  const double inv = n > 0.0 ? 1.0 / n : 0.0;
  z64* q = Q + (long)s * ldq;
  for (int i = threadIdx.x; i < npw; i += NT) q[i] = inv * b[i];
  if (threadIdx.x == 0) nrm[s] = n;
}

// Step j of the recursion for the listed systems, spread over kMsSplit
// workgroups per system (three launches, fixed-order sums).  On entry
// AQ[s][j] holds A q_j (kept: the true residuals are formed from it); on exit
// alpha_j = Re <q_j, A q_j>, w = A q_j - alpha_j q_j - beta_{j-1} q_{j-1},
// beta_j = |w| and Q[s][j+1] = w / beta_j.
constexpr int kMsSplit = 16;

__device__ __forceinline__ void ms_slice(int npw, int& i0, int& i1) {
  const int chunk = (npw + kMsSplit - 1) / kMsSplit;
  i0 = blockIdx.x * chunk;
  i1 = min(npw, i0 + chunk);
}

// part[slot][blk] = the slice's share of Re <q_j, A q_j>
__global__ void __launch_bounds__(NT)
k_ms_dot(const z64* __restrict__ Q, const z64* __restrict__ AQ, long ldq, int npw, int j,
         const int* __restrict__ act, double* __restrict__ part) {
  __shared__ double sm[NT / 64];
  const int s = act[blockIdx.y];
  int i0, i1;
  ms_slice(npw, i0, i1);
  const z64* q = Q + (long)s * ldq + (long)j * npw;
  const z64* aq = AQ + (long)s * ldq + (long)j * npw;
  double acc[1] = {0.0};
  for (int i = i0 + threadIdx.x; i < i1; i += NT) acc[0] += q[i].x * aq[i].x + q[i].y * aq[i].y;
  block_sum<double, 1>(acc, sm);
  if (threadIdx.x == 0) part[blockIdx.y * kMsSplit + blockIdx.x] = acc[0];
}

// The projection of the step's product folded in: C_v = sum over the column
// workgroups of ppart (left by the last transform), A q_j = Y - sum_v C_v
// Phi_v stored back in place, and part[slot][blk] = the slice's share of
// Re <q_j, A q_j> (what k_ms_dot leaves).
__global__ void __launch_bounds__(NT)
k_ms_proj_dot(const z64* __restrict__ Q, z64* __restrict__ AQ, long ldq, int npw, int j,
              const int* __restrict__ act, const z64* __restrict__ Phi, long ldphi, int nv,
              const z64* __restrict__ ppart, int nblk, double* __restrict__ part) {
  __shared__ double sm[NT / 64];
  __shared__ z64 C[8];
  const int slot = blockIdx.y, s = act[slot];
  if (threadIdx.x < 8) {
    z64 a{0, 0};
    if (threadIdx.x < nv)
      for (int b = 0; b < nblk; ++b) a = a + ppart[((long)slot * nblk + b) * 8 + threadIdx.x];
    C[threadIdx.x] = a;
  }
  __syncthreads();
  int i0, i1;
  ms_slice(npw, i0, i1);
  const z64* q = Q + (long)s * ldq + (long)j * npw;
  z64* aq = AQ + (long)s * ldq + (long)j * npw;
  double acc[1] = {0.0};
  for (int i = i0 + threadIdx.x; i < i1; i += NT) {
    z64 y = aq[i];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (u < nv) y = y - C[u] * Phi[(long)u * ldphi + i];
    aq[i] = y;
    acc[0] += q[i].x * y.x + q[i].y * y.y;
  }
  block_sum<double, 1>(acc, sm);
  if (threadIdx.x == 0) part[blockIdx.y * kMsSplit + blockIdx.x] = acc[0];
}

// alpha_j from the partials; w into Q[s][j+1]; part2[slot][blk] = the slice's |w|^2
__global__ void __launch_bounds__(NT)
k_ms_upd(z64* __restrict__ Q, const z64* __restrict__ AQ, long ldq, int npw, int j, const int* __restrict__ act,
         const double* __restrict__ part, double* __restrict__ part2, double* __restrict__ alpha,
         const double* __restrict__ beta, int kcap) {
  __shared__ double sm[NT / 64];
  const int slot = blockIdx.y, s = act[slot];
  double a = 0.0;
  for (int b = 0; b < kMsSplit; ++b) a += part[slot * kMsSplit + b];
  const double bp = j > 0 ? beta[(long)s * kcap + j - 1] : 0.0;
  int i0, i1;
  ms_slice(npw, i0, i1);
  const z64* q = Q + (long)s * ldq + (long)j * npw;
  const z64* aq = AQ + (long)s * ldq + (long)j * npw;
  const z64* qp = j > 0 ? q - npw : nullptr;
  z64* w = Q + (long)s * ldq + (long)(j + 1) * npw;
  double acc[1] = {0.0};
  for (int i = i0 + threadIdx.x; i < i1; i += NT) {
    z64 v = aq[i] - a * q[i];
    if (qp) v = v - bp * qp[i];
    w[i] = v;
    acc[0] += norm2(v);
  }
  block_sum<double, 1>(acc, sm);
  if (threadIdx.x == 0) {
    part2[slot * kMsSplit + blockIdx.x] = acc[0];
    if (blockIdx.x == 0) alpha[(long)s * kcap + j] = a;
  }
}

// beta_j = |w| from the partials; Q[s][j+1] = w / beta_j
__global__ void __launch_bounds__(NT)
k_ms_norm(z64* __restrict__ Q, long ldq, int npw, int j, const int* __restrict__ act,
          const double* __restrict__ part2, double* __restrict__ beta, int kcap) {
  const int slot = blockIdx.y, s = act[slot];
  double b2 = 0.0;
  for (int b = 0; b < kMsSplit; ++b) b2 += part2[slot * kMsSplit + b];
  const double bn = sqrt(b2);
  const double inv = bn > 0.0 ? 1.0 / bn : 0.0;
  int i0, i1;
  ms_slice(npw, i0, i1);
  z64* w = Q + (long)s * ldq + (long)(j + 1) * npw;
  for (int i = i0 + threadIdx.x; i < i1; i += NT) w[i] = inv * w[i];
  if (threadIdx.x == 0 && blockIdx.x == 0) beta[(long)s * kcap + j] = bn;
}

// X[s][t] = Q[s] y and the true residual r = b_s - (A - tau_t) X[s][t] =
// b_s - AQ[s] y + tau_t Q[s] y of every (system, shift), y = Y[s][.][t]
// (rows padded to ntp, a multiple of 16; grid z selects the group of 64
// shifts), AQ[s][j] = A q_j as the recursion applied it.  Rows j >= k[s] are
// never read.  On v_mfma_f64_16x16x4f64 (lane l holds A[l%16][l/16],
// B[l/16][l%16] and D[4r + l/16][l%16]) a wave computes 64 shifts x 16 plane
// waves twice (Q y and AQ y), each complex product as four real ones; |r|^2
// over the wave's 16 plane waves goes to part[(s * ntp + t) * nwt + tile].
__global__ void __launch_bounds__(256)
k_ms_combine_res(const z64* __restrict__ Q, const z64* __restrict__ AQ, long ldq, int npw,
                 const int* __restrict__ kdone, const z64* __restrict__ Y, int ldyj, int ntp, int ntau,
                 const z64* __restrict__ tau, const z64* __restrict__ B, long ldb, const int* __restrict__ bidx,
                 z64* __restrict__ X, double* __restrict__ part, int nwt) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int s = blockIdx.y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wt = blockIdx.x * 4 + w;   // 16-plane-wave tile
  const int i0 = wt * 16;
  if (i0 >= npw) return;   // no barriers below
  const int k = kdone[s];
  const z64* Qs = Q + (long)s * ldq;
  const z64* AQs = AQ + (long)s * ldq;
  const z64* Ys = Y + (long)s * ldyj * ntp;
  const int col = lane & 15, kl = lane >> 4;
  const int tb = 64 * blockIdx.z;
  const int nm = min(4, (ntp - tb) >> 4);
  const int i = i0 + col;
  d4 xr[4], xi[4], ar[4], ai[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) xr[m] = xi[m] = ar[m] = ai[m] = d4{0, 0, 0, 0};
  for (int j0 = 0; j0 < k; j0 += 4) {
    const int j = j0 + kl;
    const bool v = j < k && i < npw;
    const z64 q = v ? Qs[(long)j * npw + i] : z64{0, 0};
    const z64 aq = v ? AQs[(long)j * npw + i] : z64{0, 0};
    z64 a[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) a[m] = (j < k && m < nm) ? Ys[(long)j * ntp + tb + 16 * m + col] : z64{0, 0};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      if (m < nm) {
        xr[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m].x, q.x, xr[m], 0, 0, 0);
        xr[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[m].y, q.y, xr[m], 0, 0, 0);
        xi[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m].x, q.y, xi[m], 0, 0, 0);
        xi[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m].y, q.x, xi[m], 0, 0, 0);
        ar[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m].x, aq.x, ar[m], 0, 0, 0);
        ar[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[m].y, aq.y, ar[m], 0, 0, 0);
        ai[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m].x, aq.y, ai[m], 0, 0, 0);
        ai[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m].y, aq.x, ai[m], 0, 0, 0);
      }
    }
  }
  const z64 bv = i < npw ? B[(long)bidx[s] * ldb + i] : z64{0, 0};
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int t = tb + 16 * m + 4 * r + kl;   // one shift per 16-lane row group
      double e = 0.0;
      if (m < nm && t < ntau && i < npw) {
        const z64 x{xr[m][r], xi[m][r]};
        X[((long)s * ntau + t) * npw + i] = x;
        const z64 ta = tau[t];
        const double rx = bv.x - ar[m][r] + (ta.x * x.x - ta.y * x.y);
        const double ry = bv.y - ai[m][r] + (ta.x * x.y + ta.y * x.x);
        e = rx * rx + ry * ry;
      }
      // sum over the 16 plane waves of the row group, fixed order
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) e += __shfl_xor(e, o, 16);
      if (col == 0 && m < nm) part[((long)s * ntp + t) * nwt + wt] = e;
    }
}

// res[r] = sum_w part[r * nwt + w], in order
__global__ void __launch_bounds__(256) k_ms_res_sum(const double* __restrict__ part, int nwt, int rows,
                                                    double* __restrict__ res) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  double acc = 0.0;
  for (int w = 0; w < nwt; ++w) acc += part[(long)r * nwt + w];
  res[r] = acc;
}
}  // namespace

namespace {
// F[k][p][i] = b_p[i] / (kin[i] - e_v - z_k) + b_p[i] / (kin[i] - e_v + z_k),
// v = p mod nv; a term whose denominator vanishes is dropped
__global__ void __launch_bounds__(256)
k_model_div(const z64* __restrict__ B, int npw, const double* __restrict__ kin, const double* __restrict__ eps, int nv,
            int nb, const z64* __restrict__ zl, z64* __restrict__ F) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int p = blockIdx.y, k = blockIdx.z;
  if (i >= npw) return;
  const z64 b = B[(long)p * npw + i];
  const double d = kin[i] - eps[p % nv];
  const z64 z = zl[k];
  z64 f{0, 0};
  for (int sgn = -1; sgn <= 1; sgn += 2) {
    const double dr = d + sgn * z.x, di = sgn * z.y;   // d -+ z with sgn = -1, +1
    const double den = dr * dr + di * di;
    if (den > 0.0) f = f + z64{(b.x * dr + b.y * di) / den, (b.y * dr - b.x * di) / den};
  }
  F[((long)k * nb + p) * npw + i] = f;
}
}  // namespace

namespace {
// r = sqrt(|b|^2), ir = 1 / r, |b|^2 of system i the sum of its ns slice
// norms bb[i][0..ns) in order
__global__ void __launch_bounds__(256) k_sqrt_inv(const double* __restrict__ bb, int ns, double* __restrict__ r,
                                                  double* __restrict__ ir, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double t = 0.0;
  for (int k = 0; k < ns; ++k) t += bb[(long)i * ns + k];
  const double v = sqrt(t);
  r[i] = v;
  ir[i] = v > 0.0 ? 1.0 / v : 0.0;
}
}  // namespace

void launch_sqrt_inv(const double* bb, int ns, double* r, double* ir, int n, hipStream_t s) {
  if (n <= 0) return;
  k_sqrt_inv<<<(n + 255) / 256, 256, 0, s>>>(bb, ns, r, ir, n);
}

void launch_model_div(const z64* B, int npw, const double* kin, const double* eps, int nv, int nb, const z64* zl,
                      int nz, z64* F, hipStream_t s) {
  if (nb <= 0 || nz <= 0) return;
  k_model_div<<<dim3((npw + 255) / 256, nb, nz), 256, 0, s>>>(B, npw, kin, eps, nv, nb, zl, F);
}

void launch_ms_init(const z64* B, long ldb, const int* bidx, int npw, z64* Q, long ldq, double* nrm, int nsys,
                    hipStream_t s) {
  if (nsys <= 0) return;
  k_ms_init<<<nsys, NT, 0, s>>>(B, ldb, bidx, npw, Q, ldq, nrm);
}

int ms_step_scratch(int na) { return 2 * na * kMsSplit; }

void launch_ms_step(z64* Q, z64* AQ, long ldq, int npw, int j, const int* act, int na, double* alpha,
                    double* beta, int kcap, double* scratch, hipStream_t s, const ProjPart<double>* pp, int nblk) {
  if (na <= 0) return;
  const dim3 grid(kMsSplit, na);
  double* part = scratch;
  double* part2 = scratch + (size_t)na * kMsSplit;
  if (pp && pp->part)
    k_ms_proj_dot<<<grid, NT, 0, s>>>(Q, AQ, ldq, npw, j, act, pp->Phi, pp->ldphi, pp->nv, pp->part, nblk, part);
  else
    k_ms_dot<<<grid, NT, 0, s>>>(Q, AQ, ldq, npw, j, act, part);
  k_ms_upd<<<grid, NT, 0, s>>>(Q, AQ, ldq, npw, j, act, part, part2, alpha, beta, kcap);
  k_ms_norm<<<grid, NT, 0, s>>>(Q, ldq, npw, j, act, part2, beta, kcap);
}

int ms_res_tiles(int npw) { return (npw + 15) / 16; }

void launch_ms_combine_res(const z64* Q, const z64* AQ, long ldq, int npw, const int* kdone, const z64* Y, int ldyj,
                           int ntp, int ntau, const z64* tau, const z64* B, long ldb, const int* bidx, z64* X,
                           double* part, double* res, int nsys, hipStream_t s) {
  if (nsys <= 0 || ntau <= 0) return;
  const int nwt = ms_res_tiles(npw);
  k_ms_combine_res<<<dim3((nwt + 3) / 4, nsys, (ntp + 63) / 64), 256, 0, s>>>(Q, AQ, ldq, npw, kdone, Y, ldyj, ntp,
                                                                               ntau, tau, B, ldb, bidx, X, part, nwt);
  const int rows = nsys * ntp;
  k_ms_res_sum<<<(rows + 255) / 256, 256, 0, s>>>(part, nwt, rows, res);
}
}  // namespace lgw
