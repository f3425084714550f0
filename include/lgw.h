/* lgw — Sternheimer polarizability and Lanczos dielectric matrix on MI355X.
 *
 * C ABI of the hot path of the Lanczos/Sternheimer G0W0 scheme of
 * Laflamme Janssen, Rousseau and Cote (arXiv:1408.3036):
 *
 *   * chi0(z) applied to a potential perturbation by one Sternheimer linear
 *     system per valence band instead of a sum over conduction states
 *     (Sec. III.A: projected conjugate gradients on the squared Hermitian
 *     equation on the imaginary axis, SQMR on the two shifted equations on
 *     the real axis);
 *   * the Lanczos tridiagonalisation, with full reorthogonalisation, of the
 *     symmetrised dielectric operator eps - 1 = -v^1/2 chi0 v^1/2 (Sec. II
 *     footnote on the symmetric form, Sec. IV);
 *   * eps(z) - 1 projected on that static Lanczos basis (Sec. VI).
 *
 * Around that path: shift-Lanczos (multi-shift) solves and frequency
 * recycling (Sec. VI), the model dielectric operator (Sec. V), eps^-1 and the
 * Ritz values in the basis (Sec. IV), the correlation self-energy traces and
 * residues in the basis (Secs. II, III.B, IV, VI), adjoints of the chi0 apply
 * and of a log-det loss, a resumable Lanczos recursion, and an H application
 * that allocates nothing.
 *
 * Discretisation (the paper leaves ABINIT's conventions implicit; this is the
 * reading implemented): orthorhombic box with edges L = (Lx, Ly, Lz), a cubic
 * N^3 grid r_n = (n_x Lx, n_y Ly, n_z Lz) / N, Omega = Lx Ly Lz, dV = Omega/N^3;
 * plane waves K_m = 2 pi (m_x/Lx, m_y/Ly, m_z/Lz) with 0.5 |K_m|^2 <= ecut;
 * H = -Laplacian/2 + V_loc with V_loc applied on the grid; Coulomb kernel
 * truncated at R = min(L)/2 (Sec. IX): v(K) = 4 pi (1 - cos(K R)) / K^2,
 * v(0) = 2 pi R^2, applied on the full grid; spin factor 2.
 *
 * Memory: when opts.mem == LGW_MEM_DEVICE (default) every bulk array
 * (V_loc, psi_v, dV, dn, q0, Q, alpha, beta, E, x, y) is a device pointer on
 * the context's device; with LGW_MEM_HOST they are host pointers.  Small
 * parameter arrays (cell, grid, eps_v, z) and k_done are always host memory.
 * Grid arrays are row-major [x][y][z] (z fastest), complex values are
 * interleaved (re, im) doubles, i.e. C99 double _Complex / torch.complex128.
 * The caller owns every buffer; the library copies its inputs.
 *
 * Errors: every call returns an lgw_status.  LGW_EINVAL and LGW_ENAN from
 * argument checks leave outputs untouched.  LGW_ENOCONV / LGW_EBREAKDOWN
 * still write every output (each system holds its best iterate) and
 * lgw_get_stats tells which solves failed.  lgw_last_error gives a message.
 * A context is bound to one device and one stream and is not thread-safe.
 */
#ifndef LGW_H
#define LGW_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lgw_ctx lgw_ctx;
typedef struct { double re, im; } lgw_c128;

typedef enum { LGW_FP64 = 0, LGW_MIXED = 1 } lgw_precision;
typedef enum { LGW_MEM_DEVICE = 0, LGW_MEM_HOST = 1 } lgw_mem;
typedef enum {
  LGW_OK = 0, LGW_EINVAL = 1, LGW_ENOMEM = 2, LGW_EDEVICE = 3, LGW_ENAN = 4,
  LGW_ENOCONV = 5, LGW_EBREAKDOWN = 6
} lgw_status;

typedef struct {
  int    precision;    /* LGW_FP64 (default) or LGW_MIXED: FP32 transforms and
                          projector inside FP64 iterative refinement          */
  double tol;          /* relative residual of every Sternheimer solve
                          |b - A x| / |b|; default 1e-13                      */
  int    max_iter;     /* iterations per solve (per refinement sweep); 5000  */
  int    check_every;  /* iterations between host convergence polls; 8       */
  int    precond;      /* 0 (default): none, the unpreconditioned CG/SQMR of
                          Sec. III.  1: diagonal kinetic preconditioner,
                          applied as the symmetric scaling S = (|K|^2/2 +
                          precond_shift)^(-1/2) (squared form: S^2), so each
                          Krylov solve runs on S P A P S and x = P S y       */
  int    deterministic;/* reductions are always in a fixed order; kept for
                          interface stability                                 */
  int    mem;          /* LGW_MEM_DEVICE (default) or LGW_MEM_HOST            */
  void*  stream;       /* hipStream_t to run on; NULL = a stream the context
                          creates                                             */
  double mem_budget_gb;/* device workspace cap for batched solves; 16        */
  double inner_tol;    /* mixed mode: relative tolerance of each FP32 inner
                          solve; default 1e-5                                 */
  int    max_sweeps;   /* mixed mode: maximum FP64 refinement sweeps; 8      */
  int    use_graph;    /* 1 (default): batches of at most 64 systems replay the
                          Krylov iterations between two convergence polls as
                          a captured HIP graph                                */
  double precond_shift;/* Ha, > 0: the shift of the kinetic preconditioner; 3 */
  int    imag_form;    /* z = i*w, w > 0.  0 (default): CG on the squared form
                          ((H-e_v)^2 + w^2) y = 2 (H-e_v) b, Eq. (P2+).  1: the
                          two shifted systems (H - e_v -+ i w) g = b solved by
                          SQMR as on the real axis (Eq. (P1)); fewer H
                          applications, same chi0                             */
  int    multishift;   /* 1: a chi0 call with at least three shifts (two or
                          more frequencies) solves them all from one Lanczos
                          recursion per (column, band) on P (H - e_v) P: the
                          Krylov space is shared by every shift (H - e_v -/+ z),
                          each shift then needs a tridiagonal solve.  FP64
                          whatever the precision; every solution is checked by
                          its true residual, and those above tol are corrected
                          by the shifted solver.  0 (default): one Krylov solve
                          per shift                                           */
  int    model;        /* 1: the model dielectric operator of Sec. V (Eq.
                          (model_eq)): H -> T in the Sternheimer equations, so
                          each band solution is P (T - e_v -+ z)^-1 P b, one
                          diagonal division instead of a Krylov solve (terms
                          with a vanishing denominator are dropped).  Every
                          chi0 / Lanczos / projection call then works on
                          eps~ - 1, the second basis of Sec. V; the VJP and
                          recycling calls return EINVAL.  0 (default): H      */
  int    autotune;     /* 1 (default): the plane pass of every H application
                          uses the tile variant (threads per workgroup, LDS
                          row layout) measured fastest for this grid,
                          precision and batch size; the measurement runs once
                          per process at the first set-up with a grid (a few
                          tens of ms), and with the environment variable
                          LGW_TUNE_CACHE naming a file it is read from and
                          appended to that file.  The variants compute the
                          same transform and agree to rounding.  0: a fixed
                          variant                                             */
} lgw_opts;

/* Fill *opts with the defaults listed above. */
void lgw_default_opts(lgw_opts* opts);

/* Create a context for one system (Sec. III.A: H, the valence set).
 *   cell   [9]  lattice vectors as rows, bohr; must be diagonal (orthorhombic)
 *   grid   [3]  N, N, N: equal, one of 16, 24, 32, 40, 48, 64, 72
 *   ecut        plane-wave cut-off in Ha; the sphere must fit: max|m_i| <= N/2-1
 *   V_loc  [N^3] local potential, Ha, real
 *   n_v         valence bands, 1..32
 *   psi_v  [n_v][N^3] valence orbitals on the grid, dV sum |psi|^2 = 1,
 *               band-limited to the sphere
 *   eps_v  [n_v] (host) their energies, Ha, ascending
 *   opts        NULL for defaults
 * Checks: shapes and ranges (EINVAL), finite inputs (ENAN), then on the
 * device orthonormality of the sphere coefficients (|<i|j> - delta| <= 1e-8;
 * leakage outside the sphere shows up here) and the eigen-residual
 * |H psi_v - eps_v psi_v| <= 1e-8 Ha (EINVAL).  On error *out is NULL. */
lgw_status lgw_setup(lgw_ctx** out, const double cell[9], const int grid[3], double ecut,
                     const double* V_loc, int n_v, const lgw_c128* psi_v, const double* eps_v,
                     const lgw_opts* opts);

/* dn = chi0(z) dV for every column and frequency (Sec. III.A).
 *   dV [n_rhs][N^3]      perturbing potentials (complex allowed)
 *   z  [n_z] (host)      frequencies: (0, w) = i w on the imaginary axis
 *                        (CG on the squared equation; w = 0: CG on
 *                        (H - e_v) f = 2 P_c b); (w, eta) with w != 0: SQMR on
 *                        (H - e_v -+ (w + i eta)) g = P_c b
 *   dn [n_z][n_rhs][N^3] output, chi0(z) dV as a density (1 / bohr^3 / Ha)
 * Spin factor 2; chi0(z) x = -2 sum_v psi_v Scatter(f_v), f_v = g_- + g_+. */
lgw_status lgw_chi0_apply(lgw_ctx* ctx, int n_rhs, const lgw_c128* dV, int n_z,
                          const lgw_c128* z, lgw_c128* dn);

/* chi0_apply on several independent systems (uneven grids and band counts
 * allowed) in one call: system i applies chi0(z) of ctx[i] to its n_rhs[i]
 * columns dV[i] and writes dn[i], exactly as lgw_chi0_apply would.  Systems
 * run concurrently, each on its context's stream from its own host thread.
 * Contexts must be distinct.  Returns the worst status. */
lgw_status lgw_chi0_apply_many(int n_sys, lgw_ctx* const* ctx, const int* n_rhs,
                               const lgw_c128* const* dV, int n_z, const lgw_c128* z,
                               lgw_c128* const* dn);

/* k steps of Lanczos with full (twice classical Gram-Schmidt)
 * reorthogonalisation on M = eps(0) - 1 = -v^1/2 chi0(0) v^1/2 (Sec. IV),
 * Euclidean norm on grid values, started from q0/|q0|.
 *   alpha [k]      diagonal of T
 *   beta  [k]      beta[j] couples q_j and q_{j+1}; beta[k_done-1] is the
 *                  norm of the final residual
 *   Q     [k][N^3] Lanczos vectors q_0..q_{k-1}, or NULL
 *   k_done (host)  steps done: < k when beta < 1e-14 max|alpha| (invariant
 *                  subspace); status stays LGW_OK.  Entries past k_done are
 *                  left untouched. */
lgw_status lgw_lanczos(lgw_ctx* ctx, const lgw_c128* q0, int k, double* alpha, double* beta,
                       lgw_c128* Q, int* k_done);

/* Continues a Lanczos recursion of lgw_lanczos from a prior state (Sec. IV;
 * a recursion checkpointed after k0 steps goes on to k steps).
 *   Q     [k][N^3] in/out: rows q_0..q_{k0-1} of the prior recursion on
 *         input; rows q_0..q_{k_done-1} on return (the first k0 - 1
 *         unchanged).
 *   alpha, beta [k] in/out: entries 0..k0-1 of the prior recursion on input;
 *         entries 0..k_done-1 on return.
 * Step k0 - 1 is computed again (one chi0 application) to recover
 * q_{k0}; with the prior state as this library wrote it, the result is that
 * of one uninterrupted k-step call.  LGW_EINVAL unless 1 <= k0 <= k and the
 * prior state has beta > 0 before step k0 - 1; LGW_ENAN on non-finite
 * input.  Memory per opts.mem. */
lgw_status lgw_lanczos_resume(lgw_ctx* ctx, int k0, int k, double* alpha, double* beta, lgw_c128* Q,
                              int* k_done);

/* Block Lanczos with full reorthogonalisation on M = eps(0) - 1, the block
 * form of the Sec. IV construction: b starting vectors (rows of Q0,
 * orthonormalised first), nblk block steps, each applying M to b vectors in
 * one batched chi0 solve; M Q_j = Q_{j-1} B_{j-1}^H + Q_j A_j + Q_{j+1} B_j.
 *   b in 1..16; Q0 [b][N^3]
 *   A [nblk][b][b]  Hermitian diagonal blocks, row-major
 *   B [nblk][b][b]  upper-triangular QR factors (non-negative diagonal);
 *                   B[nblk-1] is the residual block
 *   Q [nblk*b][N^3] Lanczos vectors, or NULL
 * Each new block is orthonormalised column by column (classical
 * Gram-Schmidt twice against all previous vectors); a column whose remaining
 * norm is below 1e-10 of the block norm is replaced by a fixed-seed random
 * direction orthogonal to the basis, its row of B set to zero.  A, B are
 * always host-side-sized blocks following opts.mem. */
lgw_status lgw_block_lanczos(lgw_ctx* ctx, int b, const lgw_c128* Q0, int nblk, lgw_c128* A,
                             lgw_c128* B, lgw_c128* Q, int* nblk_done);

/* E[z] = Q^H (eps(z) - 1) Q for every z of the list (the static basis reused
 * for all frequencies, Sec. VI).  Q [k][N^3] (orthonormal rows, e.g. from
 * lgw_lanczos), E [n_z][k][k] with E[z][a][b] = <q_a, (eps(z)-1) q_b>. */
lgw_status lgw_project(lgw_ctx* ctx, int k, const lgw_c128* Q, int n_z, const lgw_c128* z,
                       lgw_c128* E);

/* Vector-Jacobian product of lgw_chi0_apply for the real scalar
 *   L = Re sum_{z,j,r} conj(g_dn[z][j](r)) dn[z][j](r),  dn[z][j] = chi0(z) dV[j]:
 *   g_dV  [n_rhs][N^3] (or NULL)  dL/d Re dV + i dL/d Im dV = sum_z chi0(conj z) g_dn[z]
 *   g_Vloc [N^3]       (or NULL)  dL/dV_loc(r), total: the valence orbitals and
 *                                  energies relax with V_loc (first-order
 *                                  perturbation theory of H = T + V_loc).
 * The V_loc part solves, per column, frequency and band, the forward and the
 * adjoint shifted systems (SQMR at z and conj z; CG at z = 0) with the
 * Sternheimer operator of Sec. III.A, then one static Sternheimer system per
 * band for the orbital response.  Outputs are overwritten.  Valence levels
 * degenerate to 1e-10 Ha contribute no rotation term (it cancels). */
lgw_status lgw_chi0_apply_vjp(lgw_ctx* ctx, int n_rhs, const lgw_c128* dV, int n_z,
                              const lgw_c128* z, const lgw_c128* g_dn, lgw_c128* g_dV,
                              double* g_Vloc);

/* lgw_lanczos followed by lgw_project on its vectors, with the projection
 * overlapped: finished Lanczos vectors are projected at all frequencies in
 * chunks (8 vectors, 16 with opts.multishift; towards the end of the
 * recursion the chunks taper to a quarter of that) by one of two worker
 * threads, each on its own stream and twin of the context (created on the
 * first call and kept with it), while the recursion continues.  The products
 * (eps(0) - 1) q_j of the recursion serve z = 0.  Outputs as lgw_lanczos
 * (alpha, beta [k], Q [k][N^3] or NULL, k_done) and lgw_project (E
 * [n_z][k][k]; with k_done < k only the leading k_done x k_done block of each
 * E[z] is written, the rest set to zero).  Needs n_z * k * N^3 complex values
 * of device workspace. */
lgw_status lgw_lanczos_project(lgw_ctx* ctx, const lgw_c128* q0, int k, int n_z, const lgw_c128* z,
                               double* alpha, double* beta, lgw_c128* Q, lgw_c128* E, int* k_done);

/* The dielectric matrix inverted within the basis (Sec. IV: eps^-1 from the
 * small matrix of the Lanczos basis instead of the full dielectric matrix).
 * For each of the n_z matrices E(z) = Q^H (eps(z) - 1) Q [k][k] (row-major,
 * as lgw_project and lgw_lanczos_project return them),
 *   Einv[z] = (I + E(z))^-1,
 * so that 1 + Q (Einv - I) Q^H is the basis approximation of eps(z)^-1
 * (exact when span(Q) is invariant under eps(z)) and Einv - I is the
 * screened factor W(z) of the self-energy traces.  Gaussian elimination
 * with partial pivoting on the host, FP64.  E and Einv [n_z][k][k] follow
 * opts.mem.  LGW_EBREAKDOWN if some I + E(z) is singular, LGW_ENAN on a
 * non-finite entry. */
lgw_status lgw_eps_inverse(lgw_ctx* ctx, int k, int n_z, const lgw_c128* E, lgw_c128* Einv);

/* Ritz values of eps(0) - 1 in the Lanczos basis (Sec. IV): the eigenvalues
 * of the k x k symmetric tridiagonal T with alpha[0..k) on the diagonal and
 * beta[0..k-1) beside it (as lgw_lanczos returns them), ascending, into
 * theta[k] (host memory).  alpha and beta follow opts.mem; beta may be NULL
 * when k = 1.  Since eps(0) - 1 is positive semidefinite they lie in
 * [0, max eigenvalue]. */
lgw_status lgw_ritz_values(lgw_ctx* ctx, int k, const double* alpha, const double* beta, double* theta);

/* Frequency recycling (Sec. VI): the static Lanczos basis of lgw_lanczos and
 * eps(i w) - 1 projected on it at imaginary frequencies without a Sternheimer
 * solve per frequency.  For every valence band the recursion's right-hand
 * sides b_{l,v} and static solutions x_{l,v}(0), with the large-frequency
 * directions P (H - e_v) b_{l,v}, span a basis gamma_v (Gram eigen-
 * decomposition, directions below 1e-7 of the largest singular value dropped,
 * then orthonormalised to rounding); H - e_v and b are expressed in it once,
 * and each imaginary-axis band solution is taken as
 * gamma 2 h (h^2 + w^2)^-1 gamma^H b with h = gamma^H (H - e_v) gamma.  The
 * result is exact at w = 0 and an approximation elsewhere (Sec. VI checks it by
 * enlarging the basis).
 *   w      [n_w]  frequencies w >= 0 of the points i*w (host memory); EINVAL
 *                 otherwise (the real axis is not recycled)
 *   alpha, beta, Q, k_done as lgw_lanczos; E [n_w][k][k] as lgw_project (the
 *          leading k_done x k_done block written, the rest zero).
 * Workspace: 2 k N_v N_pw for the captured vectors and about 6 k N_v N_pw more. */
lgw_status lgw_lanczos_recycle(lgw_ctx* ctx, const lgw_c128* q0, int k, int n_w, const double* w,
                               double* alpha, double* beta, lgw_c128* Q, lgw_c128* E, int* k_done);

/* Loss of the Lanczos-projected dielectric matrix and its gradient:
 *   L = sum_z log det(I + E(z)),  E(z) = Q^H (eps(z) - 1) Q,
 * with Q the k Lanczos vectors of eps(0) - 1 from q0 (as lgw_lanczos: the
 * static basis of Sec. IV reused for every frequency as in Sec. VI), so that
 * sum_k log(1 + theta_k(z)) over the eigenvalues of E(z).  Every z must be
 * i*w with w >= 0 (E Hermitian, I + E positive definite); otherwise EINVAL.
 *   loss   [1]   (follows opts.mem)
 *   g_Vloc [N^3] (or NULL for the loss alone) dL/dV_loc(r), overwritten; the
 *          total derivative: Q follows eps(0) through the recursion
 *          (reverse pass over the k steps with their reorthogonalisation,
 *          k - 1 further applications of eps(0) - 1), and chi0 carries the
 *          orbital response as in lgw_chi0_apply_vjp.
 *   k_done (or NULL) number of Lanczos vectors used (< k after breakdown).
 * EBREAKDOWN if some I + E(z) is not numerically positive definite. */
lgw_status lgw_lanczos_loss_vjp(lgw_ctx* ctx, const lgw_c128* q0, int k, int n_z,
                                const lgw_c128* z, double* loss, double* g_Vloc, int* k_done);

/* y = (H - shift) x on sphere coefficients (the operator inside every
 * Sternheimer solve, Sec. III.A), in the context's precision.
 *   x, y [n][npw] in the library's sphere order (lgw_sphere). */
lgw_status lgw_hpsi(lgw_ctx* ctx, int n, lgw_c128 shift, const lgw_c128* x, lgw_c128* y);

/* Correlation self-energy of state e in the dielectric basis Q (Secs. II,
 * III.B and IV; the integrand of Eq. (e_c) and its Lorentzian-model terms).
 * With s = eps_e + delta, the pair operator K = v^1/2 Phi_e f(H) Phi_e^+ v^1/2
 * (Phi_e: multiplication by psi_e) and eps^-1 - 1 inverted within span(Q),
 * W(z) = (I + E(z))^-1 - I with E(z) = Q^H (eps(z) - 1) Q:
 *   sigma_N[i]  = Re tr[W(i w_i) K_i],  f(x) = (x - s) / ((x - s)^2 + w_i^2)
 *                 (Eqs. (ge), (kge); every w from one shift-Lanczos
 *                 recursion of H per basis vector, Sec. VI),
 *   sigma_N0[i] = a^2 / (w_i^2 + a^2) Re tr[W(0) K_i]          (Eq. (g0e)),
 *   sigma_A     = Re tr[W(0) K_A],  f(x) = (a/2) / (x - s + a sgn(x - s)),
 *                 0 at x = s (Eqs. (he), (khe): the conduction states by
 *                 (H - s + a) y = P_c g on the conduction space, the valence
 *                 states by their energies).
 * The correlation energy of Eq. (e_c) is then
 * (1/pi) sum_i wt_i (sigma_N[i] - sigma_N0[i]) + sigma_A + Sigma_P for the
 * caller's quadrature (w_i, wt_i) of the half line.
 *   e      index of a valence state (0 .. n_v - 1); s must lie below every
 *          conduction state (not checked: the library knows only the
 *          valence set).
 *   alpha  Lorentzian width a > 0 (the paper uses 1 Ha).
 *   Q      [k][N^3] orthonormal basis (opts.mem layout), e.g. from lgw_lanczos.
 *   w      [n_w] imaginary frequencies > 0, host.  sigma_N, sigma_N0 [n_w]
 *          and sigma_A [1] are host memory.
 * FP64 throughout (whatever opts.precision for the resolvents of H; E(z)
 * follows the context's solver options); LGW_EINVAL for the model operator
 * (opts.model = 1) or invalid arguments; LGW_EBREAKDOWN if I + E(i w) is
 * not positive definite. */
lgw_status lgw_sigma_traces(lgw_ctx* ctx, int e, double delta, double alpha, int k, const lgw_c128* Q,
                            int n_w, const double* w, double* sigma_N, double* sigma_N0, double* sigma_A);

/* Residue term Sigma_P of Eq. (pe) for state e (Sec. VI): for every valence
 * state v with w_v = eps_v - s > 0 (weight 1; weight 1/2 at w_v = 0,
 * Theta(0) = 1/2), the element <ev*| v^1/2 (eps^-1(w_v) - 1) v^1/2 |v*e> at
 * the real frequency w_v (no broadening) from k_p Lanczos steps on
 * eps(w_v) - 1 seeded with v^1/2 |v*e>: dV |p|^2 [(I + T)^-1 - I]_00.
 *   Sigma_P = - sum_v weight_v element_v.
 * Conduction poles (states below s) are not included: s must lie below the
 * conduction band.  sigma_P [1] and n_poles [1] (or NULL) are host memory. */
lgw_status lgw_sigma_residues(lgw_ctx* ctx, int e, double delta, int k_p, double* sigma_P, int* n_poles);

/* lgw_hpsi without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same y = (H - shift) x with the same kernels and
 * precision as lgw_hpsi, its intermediates in a fixed 64 MiB device array of
 * the library (one per device, held until the process ends) instead of the
 * context's workspace.  No hipMalloc, hipFree or other allocating call is
 * made.
 *   x, y  device pointers [n][npw] (sphere order of lgw_sphere); the context
 *         must use LGW_MEM_DEVICE, else LGW_EINVAL.
 *   n     vectors.  Scratch needed, in 256-byte aligned parts: FP64
 *         16 n + 16 n N ncols bytes; mixed precision 8 n + 8 n N ncols +
 *         2 * 8 n npw bytes.  Above 64 MiB the call returns LGW_EINVAL,
 *         launches nothing, and lgw_last_error states the largest n (at
 *         silane size, 48^3 and 641 columns: 136 vectors in FP64).
 * Asynchronous: the kernels are queued on the context's stream and y is
 * complete when that stream reaches them; the call does not synchronise.
 * Every call on one device shares that device's array (nothing in it needs to
 * start at zero; the call writes everything it reads): calls that overlap on
 * one device, from any context or stream, race on it. */
lgw_status lgw_hpsi_noalloc(lgw_ctx* ctx, int n, lgw_c128 shift, const lgw_c128* x, lgw_c128* y);

/* y = v^1/2 x on grid vectors [n][N^3] (truncated Coulomb square root). */
lgw_status lgw_vhalf(lgw_ctx* ctx, int n, const lgw_c128* x, lgw_c128* y);

typedef struct { int N, npw, ncols, n_v; double omega; } lgw_info;
lgw_status lgw_get_info(const lgw_ctx* ctx, lgw_info* out);
/* Signed integer triples of the sphere in library order (host, [npw][3]). */
lgw_status lgw_sphere(const lgw_ctx* ctx, int* m);

typedef struct {
  int n_solves;             /* solves of the last chi0_apply / lanczos step */
  const int* iters;         /* [n_solves] Krylov iterations (all sweeps)    */
  const double* rel_resid;  /* [n_solves] final FP64 |b - A x| / |b|        */
  const int* refine_sweeps; /* [n_solves] FP64 refinement sweeps (mixed)    */
  const int* flags;         /* [n_solves] 1 converged, 2 breakdown, 4 max_iter */
  long long total_iters;    /* all Krylov iterations of the call            */
  long long total_happly;   /* FP64 + FP32 H applications of the call       */
} lgw_stats;
/* Views owned by the context, valid until the next call on it. */
lgw_status lgw_get_stats(const lgw_ctx* ctx, lgw_stats* out);
const char* lgw_last_error(const lgw_ctx* ctx);

/* Per-kernel timing with HIP events recorded around every batched launch
 * (more than 64 systems) on the context's stream (off by default; enabling it
 * resets the counters).
 * model_bytes is the algorithmic HBM traffic of those launches:
 *   LGW_K_PLANE_HV  xy-plane pass of H: column data read + written once, the
 *                   potential read once per launch;
 *   LGW_K_ZINV      sphere read + column write;  LGW_K_ZFWD column read +
 *                   sphere input read + sphere output written;
 *   LGW_K_PROJ      vector read (dots), read + written (update), valence
 *                   block read once;
 *   LGW_K_CG / LGW_K_SQMR  vectors touched by one update. */
enum { LGW_K_PLANE_HV = 0, LGW_K_ZINV = 1, LGW_K_ZFWD = 2, LGW_K_PROJ = 3, LGW_K_CG = 4,
       LGW_K_SQMR = 5, LGW_NKERNELS = 6,
       LGW_K_FP32 = 8 /* add to an id for the single-precision launches */ };
typedef struct { long long launches; double total_ms; double model_bytes; } lgw_timing;
lgw_status lgw_profile(lgw_ctx* ctx, int enable);
lgw_status lgw_kernel_timing(const lgw_ctx* ctx, int kernel, lgw_timing* out);
void lgw_free(lgw_ctx* ctx);

/* The plane-pass tile variant an H application of nsys systems uses in the
 * given precision (LGW_FP64, or LGW_MIXED for the single-precision inner
 * solves) on this context's grid: variant index, threads per workgroup, padded
 * LDS rows (1) or not (0), and in us[4] (or NULL) the autotuner's measured
 * microseconds per launch of each variant (zeros if not measured).  Host
 * memory; no device work. */
lgw_status lgw_tune_info(const lgw_ctx* ctx, int precision, int nsys, int* variant, int* threads, int* pad,
                         double* us);

#ifdef __cplusplus
}
#endif
#endif
