"""Pins for the CPU oracle: closed forms, invariants and brute force.

None of these compares the oracle with itself through a retyped formula: each
checks it against something the mathematics fixes independently (Lindhard
closed form, quadrature of the Coulomb kernel, matrix identities, the
spectral statements of Sec. IV, exact breakdown of Lanczos on an invariant
subspace).
"""
import numpy as np
import pytest
import scipy.integrate

from oracle.pw import Basis
from oracle.sos import SOS
from oracle import sternheimer, lindhard, lanczos
from synthetic import make_workload, random_potentials

L1, N1, E1 = 10.0, 16, 6.0


@pytest.fixture(scope="module")
def basis1():
    return Basis(L1, N1, E1)


@pytest.fixture(scope="module")
def w1():
    return make_workload(1)


@pytest.fixture(scope="module")
def sos1(basis1, w1):
    return SOS(basis1, w1.V, w1.n_v)


def _plane_wave(L, N, q):
    r = L * np.stack(np.meshgrid(*[np.arange(N)] * 3, indexing="ij"), -1).reshape(-1, 3) / N
    return np.exp(1j * (2 * np.pi / L) * r @ np.asarray(q, float))


# ---------------------------------------------------------------- discretisation
def test_sphere_count_matches_brute_force(basis1):
    assert basis1.npw == len(lindhard.sphere_triples(L1, N1, E1)) == 739


def test_scatter_of_unit_coefficient_is_normalised_plane_wave(basis1):
    j = 17
    e = np.zeros(basis1.npw, complex)
    e[j] = 1.0
    g = basis1.scatter(e)
    ref = _plane_wave(L1, N1, basis1.m[j]) / np.sqrt(basis1.omega)
    assert np.abs(g - ref).max() < 1e-14
    # grid inner product equals coefficient inner product
    rng = np.random.default_rng(0)
    c = rng.standard_normal(basis1.npw) + 1j * rng.standard_normal(basis1.npw)
    d = rng.standard_normal(basis1.npw) + 1j * rng.standard_normal(basis1.npw)
    lhs = basis1.dV * np.vdot(basis1.scatter(c), basis1.scatter(d))
    assert abs(lhs - np.vdot(c, d)) < 1e-12 * abs(np.vdot(c, d)) + 1e-12
    assert np.abs(basis1.gather(basis1.scatter(c)) - c).max() < 1e-13


def test_hamiltonian_matrix_elements_of_a_sine_potential(basis1):
    # V = A sin(2 pi x / L): Vhat(+-e_x) = -+ i A / 2, so H couples m and m +- e_x
    A = 0.7
    N = N1
    x = L1 * np.arange(N) / N
    V = A * np.sin(2 * np.pi * x / L1)[:, None, None] * np.ones((1, N, N))
    H = basis1.dense_H(V)
    pos = {tuple(m): i for i, m in enumerate(basis1.m)}
    a = pos[(0, 0, 0)]
    b = pos[(1, 0, 0)]
    # H_{ab} = Vhat(m_a - m_b) = Vhat(-e_x) = +i A/2
    assert abs(H[a, b] - 0.5j * A) < 1e-14
    assert abs(H[b, a] + 0.5j * A) < 1e-14
    assert abs(H[a, a] - 0.0) < 1e-14
    assert np.abs(H - H.conj().T).max() < 1e-14
    # matrix-free application agrees with the dense matrix
    c = np.random.default_rng(1).standard_normal(basis1.npw) + 0j
    assert np.abs(basis1.apply_H(V, c) - H @ c).max() < 1e-13


def test_truncated_coulomb_matches_quadrature():
    b = Basis(10.0, 16, 6.0)
    s = b.sqrt_coulomb()
    R = 5.0
    for flat in [0, 1, 17, 300, 2000]:
        k = np.sqrt(b.k2_grid.ravel()[flat])
        if k == 0:
            ref = scipy.integrate.quad(lambda r: 4 * np.pi * r, 0, R)[0]
        else:
            ref = scipy.integrate.quad(lambda r: 4 * np.pi * np.sin(k * r) / k, 0, R,
                                       limit=200)[0]
        assert abs(s[flat] ** 2 - ref) < 1e-10 * max(1.0, abs(ref))


# ---------------------------------------------------------------- chi0 definition
@pytest.mark.parametrize("n_v", [1, 7])
def test_sos_matches_lindhard_closed_form(basis1, n_v):
    V0 = np.zeros((N1, N1, N1))
    s = SOS(basis1, V0, n_v)
    for q in [(1, 0, 0), (2, 1, 0), (3, -2, 1), (0, 0, 0), (7, 7, 7)]:
        x = _plane_wave(L1, N1, q)
        for z in [0.0, 0.3j, 0.5 + 0.01j, -0.2 + 0.003j]:
            y = s.chi0(z, x)
            lam = lindhard.eigenvalue(L1, N1, E1, n_v, q, z)
            assert np.abs(y - lam * x).max() <= 1e-13 * max(abs(lam), 1e-2)


def test_chi0_hermitian_nsd_and_monotone_on_imaginary_axis():
    b = Basis(8.0, 12, 4.0)
    w = make_workload(1, L=8.0, N=12, ecut=4.0)
    s = SOS(b, w.V, w.n_v)
    X1 = s.chi0_matrix(0.2j)
    X2 = s.chi0_matrix(0.7j)
    for X in (X1, X2):
        assert np.abs(X - X.conj().T).max() < 1e-14 * np.abs(X).max()
        ev = np.linalg.eigvalsh(X)
        assert ev.max() <= 1e-13 * np.abs(ev).max()
    # each term -4D/(D^2 + w^2) increases towards 0 with w: X2 - X1 is PSD
    ev = np.linalg.eigvalsh(X2 - X1)
    assert ev.min() >= -1e-13 * np.abs(X1).max()
    # rank <= N_v (N_pw - N_v)
    assert s.rho.shape[0] == w.n_v * (b.npw - w.n_v)


def test_eps_minus_one_spectrum():
    b = Basis(8.0, 12, 4.0)
    w = make_workload(1, L=8.0, N=12, ecut=4.0)
    s = SOS(b, w.V, w.n_v)
    for z in [0.0, 0.4j]:
        M = s.M_matrix(z)
        ev = np.linalg.eigvalsh(0.5 * (M + M.conj().T))
        assert ev.min() >= -1e-13 * ev.max()
        one_minus_inv = np.linalg.eigvals(np.eye(M.shape[0]) - np.linalg.inv(np.eye(M.shape[0]) + M))
        assert one_minus_inv.real.min() >= -1e-12 and one_minus_inv.real.max() < 1.0


# ---------------------------------------------------------------- Sternheimer = SOS
@pytest.mark.parametrize("z", [0.0, 0.5j, 0.3 + 0.0037j, 1.2 + 0.0037j, -0.4 + 0.02j])
def test_dense_sternheimer_equals_sum_over_states(basis1, w1, sos1, z):
    x = random_potentials(N1, 1, 11, real=False)[0]
    y1 = sos1.chi0(z, x)
    y2 = sternheimer.dense_chi0(basis1, w1.V, w1.psi, w1.eps, complex(z), x)
    assert np.linalg.norm(y1 - y2) <= 1e-12 * np.linalg.norm(y1)


def test_squared_form_equals_sum_of_shifted_solves(basis1, w1):
    # Sec. III.A: the squared imaginary-axis equation returns f_+ + f_-
    H = basis1.dense_H(w1.V)
    H = 0.5 * (H + H.conj().T)
    U = sternheimer._valence_conj(basis1, w1.psi)
    Pv = U.T @ U.conj()
    Pc = np.eye(basis1.npw) - Pv
    I = np.eye(basis1.npw)
    x = random_potentials(N1, 1, 12)[0]
    w = 0.37
    for v in range(w1.n_v):
        b = Pc @ basis1.gather(w1.psi[v].conj() * x)
        A = H - w1.eps[v] * I
        fsq = np.linalg.solve(Pc @ (A @ A + w * w * I) @ Pc + Pv, 2 * Pc @ A @ b)
        fp = np.linalg.solve(Pc @ (A + 1j * w * I) @ Pc + Pv, b)
        fm = np.linalg.solve(Pc @ (A - 1j * w * I) @ Pc + Pv, b)
        assert np.linalg.norm(fsq - (fp + fm)) <= 1e-12 * np.linalg.norm(fsq)


@pytest.mark.parametrize("z", [0.0, 0.5j, 0.3 + 0.0037j])
def test_matrix_free_sternheimer_equals_sum_over_states(basis1, w1, sos1, z):
    x = random_potentials(N1, 1, 13)[0]
    mf = sternheimer.MatrixFree(basis1, w1.V, w1.psi, w1.eps)
    y1 = sos1.chi0(z, x)
    y3 = mf.chi0(complex(z), x)
    assert np.linalg.norm(y1 - y3) <= 1e-11 * np.linalg.norm(y1)


def test_large_frequency_limit(basis1, w1, sos1):
    # Sec. VI: x(iw) -> (H - e_v) b / w^2, so w^2 chi0(iw) x -> -4 sum_v psi_v Scatter((H-e_v) b_v)
    x = random_potentials(N1, 1, 14)[0]
    U = sternheimer._valence_conj(basis1, w1.psi)
    lim = np.zeros(N1 ** 3, complex)
    for v in range(w1.n_v):
        g = basis1.gather(w1.psi[v].conj() * x)
        b = g - U.T @ (U.conj() @ g)
        hb = basis1.apply_H(w1.V, b) - w1.eps[v] * b
        hb = hb - U.T @ (U.conj() @ hb)
        lim += -4 * w1.psi[v] * basis1.scatter(hb)
    errs = []
    for w in [200.0, 400.0, 800.0]:
        y = w ** 2 * sos1.chi0(1j * w, x)
        errs.append(np.linalg.norm(y - lim) / np.linalg.norm(lim))
    assert errs[2] < 1e-3
    # O(1/w^2) decay: doubling w divides the error by ~4
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_generator_ground_state_is_oracle_valence_space(basis1, w1, sos1):
    C = basis1.gather(w1.psi)                       # [n_v, npw]
    H = basis1.dense_H(w1.V)
    for v in range(w1.n_v):
        assert np.linalg.norm(H @ C[v] - w1.eps[v] * C[v]) < 1e-10
    assert np.allclose(sos1.eps[:w1.n_v], w1.eps, atol=1e-12)
    # same subspace: projector difference
    Cv = sos1.C[:, :w1.n_v]
    P1 = Cv @ Cv.conj().T
    P2 = C.T @ C.conj()
    assert np.abs(P1 - P2).max() < 1e-11


# ---------------------------------------------------------------- Lanczos
@pytest.fixture(scope="module")
def small_M():
    b = Basis(8.0, 12, 4.0)
    w = make_workload(1, L=8.0, N=12, ecut=4.0)
    s = SOS(b, w.V, w.n_v)
    M = s.M_matrix(0.0)
    return b, s, 0.5 * (M + M.conj().T)


def test_lanczos_invariants(small_M):
    b, s, M = small_M
    q0 = random_potentials(b.N, 1, 21)[0]
    k = 30
    a, be, Q, kd = lanczos.lanczos(lambda v: M @ v, q0, k)
    assert kd == k
    assert np.abs(Q.conj() @ Q.T - np.eye(k)).max() < 1e-13
    T = lanczos.tridiag(a, be)
    nrm = np.linalg.norm(M, 2)
    assert np.abs(Q.conj() @ M @ Q.T - T).max() < 1e-12 * nrm
    # M Q - Q T = beta_k q_k e_k^T : residual only in the last column, of norm beta_k
    R = M @ Q.T - Q.T @ T
    assert np.abs(R[:, :-1]).max() < 1e-12 * nrm
    assert abs(np.linalg.norm(R[:, -1]) - be[-1]) < 1e-12 * nrm
    # Ritz values inside the spectrum, largest converged first
    lam = np.linalg.eigvalsh(M)
    th = np.linalg.eigvalsh(T)
    assert th.min() >= lam.min() - 1e-12 * nrm and th.max() <= lam.max() + 1e-12 * nrm
    assert abs(th[-1] - lam[-1]) < 1e-8 * lam[-1]
    assert abs(th[0] - lam[0]) > abs(th[-1] - lam[-1])


def test_lanczos_spans_monomial_krylov_space(small_M):
    b, s, M = small_M
    q0 = random_potentials(b.N, 1, 22)[0]
    k = 5
    _, _, Q, _ = lanczos.lanczos(lambda v: M @ v, q0, k)
    K = [q0 / np.linalg.norm(q0)]
    for _ in range(k - 1):
        K.append(M @ K[-1])
    Qk, _ = np.linalg.qr(np.array(K).T)
    # both orthonormal bases span the same space: singular values of Qk^H Q are 1
    sv = np.linalg.svd(Qk.conj().T @ Q.T, compute_uv=False)
    assert np.abs(sv - 1).max() < 1e-9


def test_lanczos_breaks_down_on_two_plane_wave_seed(basis1):
    # V = 0: eps - 1 is diagonal in plane waves with eigenvalue -v(K_q) lambda(q, 0)
    V0 = np.zeros((N1, N1, N1))
    s = SOS(basis1, V0, 1)
    q1, q2 = (1, 0, 0), (0, 2, 1)
    seed = _plane_wave(L1, N1, q1) + 0.5 * _plane_wave(L1, N1, q2)
    a, be, Q, kd = lanczos.lanczos(lambda v: s.M(0.0, v), seed, 6)
    assert kd == 2
    th = np.sort(np.linalg.eigvalsh(lanczos.tridiag(a, be)))
    R = L1 / 2
    ref = []
    for q in (q1, q2):
        k = 2 * np.pi / L1 * np.linalg.norm(q)
        v = 4 * np.pi * (1 - np.cos(k * R)) / k ** 2
        ref.append(-v * lindhard.eigenvalue(L1, N1, E1, 1, q, 0.0).real)
    assert np.allclose(th, np.sort(ref), rtol=1e-12)


def test_projected_eps_at_zero_is_the_tridiagonal(small_M):
    b, s, M = small_M
    q0 = random_potentials(b.N, 1, 23)[0]
    a, be, Q, _ = lanczos.lanczos(lambda v: s.M(0.0, v), q0, 6)
    E = lanczos.project(lambda z, v: s.M(z, v), Q, [0.0, 0.5j])
    assert np.abs(E[0] - lanczos.tridiag(a, be)).max() < 1e-12 * np.abs(a).max()
    # eps(iw) - 1 decreases along iw (Sec. VI): E(0.5i) <= E(0) in the Loewner order
    assert np.linalg.eigvalsh(E[0] - E[1]).min() > -1e-13


def test_logdet_loss_depends_only_on_the_krylov_space(small_M):
    # The loss is invariant under any unitary change of basis of span(Q), so an
    # orthonormal basis of the monomial Krylov space {q, Mq, ..., M^{k-1} q}
    # from a QR factorisation, with dense eps(z) - 1 matrices, must give it too.
    b, s, M = small_M
    q0 = random_potentials(b.N, 1, 24)[0]
    k, zs = 4, [0.0, 0.3j, 1.5j]
    L = lanczos.logdet_loss(lambda z, v: s.M(z, v), q0, k, zs)
    K = [q0 / np.linalg.norm(q0)]
    for _ in range(k - 1):
        K.append(M @ K[-1])
    U, _ = np.linalg.qr(np.array(K).T)
    ref = 0.0
    for z in zs:
        Mz = s.M_matrix(z)
        E = U.conj().T @ (0.5 * (Mz + Mz.conj().T)) @ U
        ref += np.sum(np.log1p(np.linalg.eigvalsh(E)))
    assert abs(L - ref) < 1e-9 * abs(ref)
    # at z = 0 alone the projected matrix is the Lanczos tridiagonal
    a, be, _, _ = lanczos.lanczos(lambda v: s.M(0.0, v), q0, k)
    T = lanczos.tridiag(a, be)
    L0 = lanczos.logdet_loss(lambda z, v: s.M(z, v), q0, k, [0.0])
    assert abs(L0 - np.linalg.slogdet(np.eye(k) + T)[1]) < 1e-12 * abs(L0)


# ---------------------------------------------------------------- block Lanczos
def test_block_lanczos_with_one_vector_is_lanczos(small_M):
    b, s, M = small_M
    q0 = random_potentials(b.N, 1, 31)[0]
    a, be, Q, _ = lanczos.lanczos(lambda v: M @ v, q0, 10)
    A, B, QB = lanczos.block_lanczos(lambda v: M @ v, q0[None], 10)
    assert np.allclose(A[:, 0, 0].real, a, atol=1e-12 * np.abs(a).max())
    assert np.allclose(B[:, 0, 0].real, be, atol=1e-12 * np.abs(a).max())
    # same vectors up to a unit phase per vector
    ph = np.sum(Q.conj() * QB, axis=1)
    assert np.allclose(np.abs(ph), 1.0, atol=1e-10)


def test_block_lanczos_invariants(small_M):
    b, s, M = small_M
    Q0 = random_potentials(b.N, 4, 32)
    A, B, Q = lanczos.block_lanczos(lambda v: M @ v, Q0, 6)
    k = Q.shape[0]
    assert k == 24
    assert np.abs(Q.conj() @ Q.T - np.eye(k)).max() < 1e-13
    T = lanczos.block_tridiag(A, B)
    nrm = np.linalg.norm(M, 2)
    assert np.abs(Q.conj() @ M @ Q.T - T).max() < 1e-12 * nrm
    # R_0-free start: the first block spans the starting vectors
    sv = np.linalg.svd(Q[:4].conj() @ (Q0 / np.linalg.norm(Q0, axis=1, keepdims=True)).T,
                       compute_uv=False)
    assert np.all(sv > 1e-8)
    # block Krylov span: span(Q) = span{Q0, M Q0, M^2 Q0, ...} (first 3 blocks)
    K = [Q0.T]
    for _ in range(2):
        K.append(M @ K[-1])
    Kq, _ = np.linalg.qr(np.concatenate(K, axis=1))
    sv = np.linalg.svd(Kq.conj().T @ Q[:12].T, compute_uv=False)
    assert np.abs(sv - 1).max() < 1e-8
    # B_j upper triangular with non-negative diagonal
    for Bj in B:
        assert np.abs(np.tril(Bj, -1)).max() == 0.0
        assert np.all(np.diag(Bj).real >= 0)
