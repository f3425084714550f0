// Host-side launchers of the lgw HIP kernels.  All pointers are device
// pointers; every launch goes to the given stream.  Grid vectors are stored
// plane-major ([z][x][y], "zxy"), sphere vectors in the column order of Geom,
// z-column intermediates as [z][col].
#pragma once
#include "common.h"

namespace lgw {

constexpr int kMaxBands = 32;   // bands handled by the projector kernels

// Projector partial sums that the CG kernels of a small batch leave for the
// next operator application, which then skips the projector's dot products
// and forms the projected input in its first transform (launch_zinv_fed):
// part[k][sys][v] = sum over slice k of conj(Phi_v) (pre .* p_sys), with the
// slices of the split CG kernels (the initialisation writes slice 0 with the
// whole sum and zeroes the others).  part == null: no partial sums.
template <typename T>
struct ProjFeed {
  const cplx<T>* Phi = nullptr;   // [nv][ldphi]
  long ldphi = 0;
  int nv = 0;
  const T* pre = nullptr;         // scaling applied before the projection, or null
  cplx<T>* part = nullptr;        // [nsplit][ntot][nv]
  int ntot = 0;                   // systems of the batch (stride of part)
  int nsplit = 1;
  // Direction update in the first transform (small preconditioned CG
  // batches, see launch_cg_step_fed): with r != null, part holds the slice sums of the
  // residual r, and while theta[sys] >= 0 the transform first sets
  // p = r + beta p (beta = theta / rr) and uses C = sum(part) + beta Cp;
  // its workgroup 0 leaves C in Cn (the last transform moves it to Cp).
  // With r set, the direction D given to the transform must be p.
  const cplx<T>* r = nullptr;
  cplx<T>* p = nullptr;           // the directions, updated in place
  const T* rr = nullptr;
  const T* theta = nullptr;
  const cplx<T>* Cp = nullptr;    // [ntot][nv] coefficients of the current p
  cplx<T>* Cn = nullptr;          // [ntot][nv] those of the new p
};

bool grid_supported(int N);

// Projector coefficients formed by the last transform (zfwd) as it stores
// Y: part[(slot * nblk + blk) * 8 + v] = sum over the column workgroup blk
// of conj(Phi_v) Y, v < nv <= 8 (nblk = zcol_blocks(g)); the multi-shift step
// then applies Y - Phi C with C the sum of the blocks.  part == null: off.
template <typename T>
struct ProjPart {
  const cplx<T>* Phi = nullptr;
  long ldphi = 0;
  int nv = 0;
  cplx<T>* part = nullptr;
};

// CG step work done by the last transform of an operator application: per
// column workgroup k of active slot j, part[j * nblk + k] = the block's
// Re p^H y of its store y with the given vectors p (the directions where the
// store is the final A p, the projected input P S p where an outer projection
// follows: p^H S P y = (P S p)^H y); workgroup 0 also commits the norm parked
// in theta to rr (theta >= 0), as the split CG's first phase would.
// part == null: off.
template <typename T>
struct CgDot {
  const cplx<T>* p = nullptr;   // directions, ld ldp
  long ldp = 0;
  T* part = nullptr;            // [nslots][nblk], nblk = zcol_blocks(g)
  T* rr = nullptr;
  T* theta = nullptr;
  // direction update in the first transform (ProjFeed::r): workgroup 0 also
  // moves the new direction's projector coefficients Cn to Cp
  cplx<T>* Cp = nullptr;
  const cplx<T>* Cn = nullptr;
  int nv = 0;
};

// ---- transforms (T = double or float) -----------------------------------
// sphere -> columns: Tb[z][c] = scale * IFFT_z(X column c)
template <typename T>
void launch_zinv(const Geom& g, const cplx<T>* tw, const cplx<T>* X, long ldx,
                 cplx<T>* Tb, long ldt, T scale, const int* act, int nsys, hipStream_t s);
// the same pass (scale 1) on the projected input X = P (f.pre .* D), formed on
// the fly from the direction D and the partial sums in f.part (ProjFeed):
// X = f.pre .* D - sum_v Phi_v C_v with C_v the sum of the slices; X is also
// written to Xout (the same layout as D, ld ldx)
template <typename T>
void launch_zinv_fed(const Geom& g, const cplx<T>* tw, const ProjFeed<T>& f, const cplx<T>* D, cplx<T>* Xout,
                     long ldx, cplx<T>* Tb, long ldt, const int* act, int nsys, hipStream_t s);
// middle pass of H: Tb <- FFT_xy(Vt[z] * IFFT_xy(Tb)) on every z plane (unscaled)
template <typename T>
void launch_plane_hv(const Geom& g, const cplx<T>* tw, cplx<T>* Tb, long ldt, const T* Vt,
                     const int* act, int nsys, hipStream_t s, int variant);
// tile variants of the plane pass: count, and (threads, padded rows) of one
int plane_variants();
void plane_variant_shape(int N, int v, int* threads, int* pad);
// columns -> sphere: Y = scale * FFT_z(Tb) [+ (kin - shift[sys]) X] [+ ecoef[sys] E]
template <typename T>
void launch_zfwd(const Geom& g, const cplx<T>* tw, const cplx<T>* Tb, long ldt, T scale,
                 const cplx<T>* X, long ldx, const cplx<T>* shift,
                 const cplx<T>* E, long lde, const T* ecoef,
                 cplx<T>* Y, long ldy, const int* act, int nsys, hipStream_t s,
                 const T* dout = nullptr,     // optional per-plane-wave scaling of Y
                 const CgDot<T>& cd = {},     // optional CG dot products (CgDot)
                 const ProjPart<T>* pp = nullptr);   // optional projector coefficients (ProjPart)
// column workgroups of the column passes (one run of the sphere vector each)
int zcol_blocks(const Geom& g);
// Tb[j*nv+v][z][c] = FFT_xy(U[v][z] * X[j][z]) at the column positions (unscaled)
template <typename T>
void launch_plane_pair_fwd(const Geom& g, const cplx<T>* tw, const cplx<T>* U, int nv,
                           const cplx<T>* X, long ldx, int nj, cplx<T>* Tb, long ldt,
                           hipStream_t s);
// out[j][z] (+)= coef * sum_v Psi[v][z] * IFFT_xy(Tb[j*nv+v][z] placed at columns)
template <typename T>
void launch_plane_acc(const Geom& g, const cplx<T>* tw, const cplx<T>* Tb, long ldt,
                      const cplx<T>* Psi, int nv, cplx<T>* out, long ldo, T coef, int nj,
                      bool accumulate, hipStream_t s);
// full 2D transform of every z plane of nvec grid vectors, in place, or from
// src (same layout, not overlapping G) into G
template <typename T>
void launch_plane_full(int N, const cplx<T>* tw, cplx<T>* G, long ldg, int nvec, int sign,
                       hipStream_t s, const cplx<T>* src = nullptr);
// every z-line of nvec grid vectors: G <- IFFT_z(scale * mul * FFT_z(G))
template <typename T>
void launch_zfull_mul(int N, const cplx<T>* tw, cplx<T>* G, long ldg, const T* mul, T scale,
                      int nvec, hipStream_t s);

// ---- layout -------------------------------------------------------------
// out[v][z][x][y] = (conj? conj : id)(in[v][x][y][z]) (and the inverse)
void launch_xyz_to_zxy(int N, const z64* in, long ldi, z64* out, long ldo, int nvec, bool conj_in,
                       hipStream_t s);
void launch_zxy_to_xyz(int N, const z64* in, long ldi, z64* out, long ldo, int nvec,
                       hipStream_t s);
void launch_real_xyz_to_zxy(int N, const double* in, double* out, hipStream_t s);
void launch_real_zxy_to_xyz(int N, const double* in, double* out, hipStream_t s);

// ---- projector and solvers ----------------------------------------------
// Y <- Y - Phi (Phi^H Y) for every listed system
template <typename T>
void launch_proj(const cplx<T>* Phi, long ldphi, int nv, int npw, cplx<T>* Y, long ldy,
                 const int* act, int nsys, hipStream_t s);

enum : int { FLAG_CONV = 1, FLAG_BREAK = 2, FLAG_MAXIT = 4 };

template <typename T>
struct SolveVecs {
  cplx<T>* x; cplx<T>* r; cplx<T>* p; cplx<T>* Ap; cplx<T>* d;  // d only for SQMR
  long ld;
  T* rr;          // CG: r^H r      SQMR: tau
  T* bb;          // |b|^2
  T* theta;       // SQMR theta
  cplx<T>* rho;   // SQMR rho
  int* flag;
  int* iters;
  int* cnt;       // ticket counters per active slot, zero between launches (fed CG kernels), or null
};
// With f.part: the split-grid initialisation of a small preconditioned batch,
// which also leaves the first projection's slice sums and needs v.cnt (zero)
// and npart (nsys * f.nsplit entries)
template <typename T>
void launch_cg_init(const SolveVecs<T>& v, const cplx<T>* b, long ldb, const int* bidx, int npw,
                    int nsys, bool keep_x, const int* act, hipStream_t s, const ProjFeed<T>& f = {},
                    T* npart = nullptr);
template <typename T>
void launch_cg_step(const SolveVecs<T>& v, int npw, T tol2, const int* act, int nsys, hipStream_t s);
template <typename T>
void launch_sqmr_init(const SolveVecs<T>& v, const cplx<T>* b, long ldb, const int* bidx, int npw,
                      int nsys, bool keep_x, const int* act, hipStream_t s);
template <typename T>
void launch_sqmr_step(const SolveVecs<T>& v, int npw, T tol, const int* act, int nsys, hipStream_t s);

// res[sys] = |b[bidx[sys]] - AX[sys]|^2, optionally R[sys] = b - AX
template <typename T>
void launch_resid(const cplx<T>* b, long ldb, const int* bidx, const cplx<T>* AX, long lda,
                  cplx<T>* R, long ldr, double* res, int npw, const int* act, int nsys,
                  hipStream_t s);
// the same over ns workgroups per system: res[sys * ns + k] is the norm of
// slice k (the caller sums them)
template <typename T>
void launch_resid_split(const cplx<T>* b, long ldb, const int* bidx, const cplx<T>* AX, long lda, cplx<T>* R,
                        long ldr, double* res, int ns, int npw, const int* act, int nsys, hipStream_t s);

// ---- BLAS-1 style helpers on long vectors --------------------------------
// out[i*m + j]... generic dot products: h[i] = sum_e conj(A[i][e]) w[e], i < m
void launch_dots(const z64* A, long lda, int m, const z64* w, long n, z64* h, z64* partial,
                 hipStream_t s);
// w -= sum_i A[i] h[i]
void launch_gemv_sub(const z64* A, long lda, int m, const z64* h, z64* w, long n, hipStream_t s);
// scalar Lanczos helpers (device scalars)
void launch_lanczos_alpha(const z64* q, const z64* w, long n, double* alpha_j, z64* partial,
                          hipStream_t s);
// one classical Gram-Schmidt pass: w = in - A (A^H in) over the m rows of A,
// in = src (not overlapping w) or w itself; re_last (or null) receives
// Re <A_{m-1}, in>.  h [m] and partial [m * 64] are workspace.
void launch_cgs_pass(const z64* A, long lda, int m, z64* w, const z64* src, long n, z64* h, z64* partial,
                     double* re_last, hipStream_t s);
// w = src - alpha_j q - beta_prev qprev (src null: w itself)
void launch_lanczos_sub(z64* w, const z64* q, const z64* qprev, const double* alpha_j, const double* beta_prev,
                        long n, hipStream_t s, const z64* src = nullptr);
// out = |w|; with pair (and alpha), also pair[0] = *alpha, pair[1] = |w|
void launch_norm(const z64* w, long n, double* out, z64* partial, hipStream_t s, const double* alpha = nullptr,
                 double* pair = nullptr);
void launch_scale_into(const z64* w, const double* nrm, z64* q, long n, hipStream_t s);
void launch_axpby(z64* y, const z64* x, z64 a, z64 b, long n, hipStream_t s);
void launch_add(z64* y, const z64* a, const z64* b, long n, hipStream_t s);
// y = a .* b (elementwise)
void launch_mul(z64* y, const z64* a, const z64* b, long n, hipStream_t s);
// any non-finite value -> *flag = 1
void launch_finite_check(const double* x, long n, int* flag, hipStream_t s);
// mixed precision conversions
void launch_cvt_64_32(const z64* in, z32* out, long n, hipStream_t s);
void launch_cvt_32_64(const z32* in, z64* out, long n, hipStream_t s);
// p[0..n) = v (a fill kernel: no memset node, so it can sit in a captured graph)
template <class T>
void launch_fill(cplx<T>* p, cplx<T> v, long n, hipStream_t s);
// x[sys] += scale[sys] * (d .* e[sys]), d (per plane wave, single precision)
// optional; assign: x[sys] = scale[sys] * (d .* e[sys])
void launch_cvt_32_64_axpy(const z32* e, z64* x, const double* scale, const int* sys_of_vec,
                           long ld, int npw, int nsys, hipStream_t s, const float* d = nullptr,
                           bool assign = false);

}  // namespace lgw

namespace lgw {
void launch_rows_out(const z64* src, long lds, z64* dst, long ldd, const int* didx, const int* a, const int* b,
                     int n, int np, hipStream_t s);
// out[sys] = d .* single(scale[sys] * in[sys]), d (per plane wave) optional
void launch_scale_cvt(const z64* in, long ldi, z32* out, long ldo, const double* scale, const int* act, int n,
                      int nsys, hipStream_t s, const float* d = nullptr);
void launch_gemm_hn(const z64* A, long lda, int m, const z64* B, long ldb, int p, long n, z64* C, z64* partial,
                    hipStream_t s);
// Y[yrow] = d .* X[xrow] for nrows rows (xrow = xi ? xi[i] : i, same for yrow)
template <typename T>
void launch_scale_diag(const cplx<T>* X, long ldx, const int* xi, cplx<T>* Y, long ldy, const int* yi, const T* d,
                       int n, int nrows, hipStream_t s);
}  // namespace lgw

namespace lgw {
// Y <- Y - Phi (Phi^H Y) with the dots on the matrix cores; part needs
// proj_ksplit(npw, nsys) * nsys * nv entries of workspace.
template <typename T> int proj_ksplit(int npw, int nsys);
template <typename T>
void launch_proj_mfma(const cplx<T>* Phi, long ldphi, int nv, int npw, cplx<T>* Y, long ldy, const int* act,
                      int nsys, cplx<T>* part, hipStream_t s);
// Y = dpost .* P (dpre .* X) (X may be Y; null scalings are 1)
template <typename T>
void launch_proj_mfma(const cplx<T>* Phi, long ldphi, int nv, int npw, const cplx<T>* X, cplx<T>* Y, long ldy,
                      const int* act, int nsys, cplx<T>* part, const T* dpre, const T* dpost, hipStream_t s);
}  // namespace lgw

namespace lgw {
// W[c] -= sum_{i<m} X[i] Cm[c*m + i], c < b
void launch_block_sub(z64* W, long ldw, int b, const z64* X, long ldx, int m, const z64* Cm, long n,
                      hipStream_t s);
}  // namespace lgw

namespace lgw {
// out[e] += Re(c * conj(a[e]) * b[e])
void launch_acc_re(double* out, const z64* a, const z64* b, z64 c, long n, hipStream_t s);
void launch_conj(const z64* in, z64* out, long n, hipStream_t s);
}  // namespace lgw

namespace lgw {
// CG update spread over nsplit workgroups per system (small batches); part
// needs 2 * nsys * nsplit entries
template <typename T>
void launch_cg_step_split(const SolveVecs<T>& v, int npw, T tol2, const int* act, int nsys, int nsplit, T* part,
                          hipStream_t s);
// The rest of a preconditioned small-batch CG step when the transforms do the direction
// update (ProjFeed::r) and p^H A p (CgDot): x += alpha p, r -= alpha A p, the
// slice sums of the new r for the next projection, and, by the last workgroup
// of each system to finish (an atomic ticket on v.cnt), the new norm parked in
// theta, the count and the convergence flag.  part needs nsys * nsplit entries.
template <typename T>
void launch_cg_step_fed(const SolveVecs<T>& v, int npw, T tol2, const int* act, int nsys, int nsplit, T* part,
                        const T* dots, int ndots, const ProjFeed<T>& f, hipStream_t s);
}  // namespace lgw

namespace lgw {
// Multi-shift Lanczos: Q rows of system s at Q + s * ldq (k vectors of npw);
// alpha/beta [nsys][kcap]; Y [nsys][ntau][kcap]
// r = sqrt(bb), ir = 1 / r (0 where bb = 0)
// r = |b|, ir = 1/|b| (0 for a zero b) from the ns slice norms per system bb[n][ns]
void launch_sqrt_inv(const double* bb, int ns, double* r, double* ir, int n, hipStream_t s);
// model operator (H -> T): F[k][p] = B[p] / (kin - e_{p mod nv} - z_k) + B[p] / (kin - e_{p mod nv} + z_k),
// terms with a vanishing denominator dropped
void launch_model_div(const z64* B, int npw, const double* kin, const double* eps, int nv, int nb, const z64* zl,
                      int nz, z64* F, hipStream_t s);
void launch_ms_init(const z64* B, long ldb, const int* bidx, int npw, z64* Q, long ldq, double* nrm, int nsys,
                    hipStream_t s);
// scratch needs ms_step_scratch(na) doubles.  With pp (projector
// coefficients the last transform left over nblk column workgroups), AQ[s][j]
// holds the unprojected product on entry and is projected in place first.
int ms_step_scratch(int na);
void launch_ms_step(z64* Q, z64* AQ, long ldq, int npw, int j, const int* act, int na, double* alpha,
                    double* beta, int kcap, double* scratch, hipStream_t s, const ProjPart<double>* pp = nullptr,
                    int nblk = 0);
// X[s][t] = Q[s] y and res[s * ntp + t] = |b - AQ[s] y + tau_t X[s][t]|^2 with
// y = Y[s][.][t], b = B[bidx[s]]; part needs nsys * ntp * ms_res_tiles(npw)
// entries (rows t >= ntau of res are zero)
int ms_res_tiles(int npw);
void launch_ms_combine_res(const z64* Q, const z64* AQ, long ldq, int npw, const int* kdone, const z64* Y, int ldyj,
                           int ntp, int ntau, const z64* tau, const z64* B, long ldb, const int* bidx, z64* X,
                           double* part, double* res, int nsys, hipStream_t s);
// C[b][a] = sum_e conj(A[a][e]) B[b][e] for a < m, b < p, on the matrix cores;
// partial needs gemm_hn_slices(n, p) * min(m, 64) * p entries
int gemm_hn_slices(long n, int p);
void launch_gemm_hn_mfma(const z64* A, long lda, int m, const z64* B, long ldb, int p, long n, z64* C, z64* partial,
                         hipStream_t s);
}  // namespace lgw
