"""Pins of the frequency-recycling oracle (Sec. VI, oracle/recycle.py) against
what the mathematics fixes: exactness at zero frequency, exactness when the
basis is the whole conduction space or an invariant subspace holding the
right-hand side (dense spectral formula), the SVD basis itself, and the
accuracy check the paper describes (adding a finite-frequency solution to the
basis)."""
import numpy as np
import pytest

from oracle import lanczos as olz
from oracle.pw import Basis
from oracle.recycle import band_rhs, gamma_basis, projected_h, recycled_E, solve_in_basis
from oracle.sternheimer import MatrixFree
from synthetic import make_workload, random_potentials


@pytest.fixture(scope="module")
def c1():
    w = make_workload(1)
    b = Basis(w.L, w.N, w.ecut)
    mf = MatrixFree(b, w.V, w.psi, w.eps)
    q0 = random_potentials(w.N, 1, 91)[0]
    _, _, Q, _ = olz.lanczos(lambda x: mf.M(0.0, x), q0, 5)
    return w, b, mf, Q


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_zero_frequency_is_exact(c1):
    """x(0) lies in every band's basis, and h is the Galerkin matrix of H - e_v,
    so the recycled static block equals the directly projected one."""
    _, _, mf, Q = c1
    E_rec = recycled_E(mf, Q, [0.0])
    E = olz.project(mf.M, Q, [0.0])
    assert _rel(E_rec, E) < 1e-10


def test_full_conduction_basis_is_exact_at_every_frequency(c1):
    """With the whole conduction space as the basis the small problem is the
    full one: the imaginary-axis blocks match the direct projection."""
    _, b, mf, Q = c1
    P = np.eye(b.npw) - mf.U.T @ mf.U.conj()
    ev, vecs = np.linalg.eigh(0.5 * (P + P.conj().T))
    G = vecs[:, ev > 0.5].T.copy()
    assert G.shape[0] == b.npw - len(mf.eps_v)
    ws = [0.3, 1.0, 3.0]
    E_rec = recycled_E(mf, Q, ws, bases=[G] * len(mf.eps_v))
    E = olz.project(mf.M, Q, [1j * x for x in ws])
    assert _rel(E_rec, E) < 1e-9


def test_invariant_subspace_reproduces_the_spectral_formula(c1):
    """A basis of eigenvectors of P(H - e_v)P holding b: the small-matrix
    solution equals 2 sum_k lam_k / (lam_k^2 + w^2) <u_k, b> u_k."""
    w, b, mf, _ = c1
    v = 1
    H = b.dense_H(w.V)
    H = 0.5 * (H + H.conj().T)
    P = np.eye(b.npw) - mf.U.T @ mf.U.conj()
    A = P @ (H - mf.eps_v[v] * np.eye(b.npw)) @ P
    lam, U = np.linalg.eigh(0.5 * (A + A.conj().T))
    cond = np.flatnonzero(np.abs(np.diag(U.conj().T @ P @ U)) > 0.5)[[0, 3, 7, 20, 50, 200]]
    G = U[:, cond].T.copy()
    rng = np.random.default_rng(5)
    rhs = G.T @ (rng.standard_normal(len(cond)) + 1j * rng.standard_normal(len(cond)))
    h = projected_h(mf, v, G)
    for om in (0.0, 0.4, 2.5):
        f = G.T @ solve_in_basis(h, G.conj() @ rhs, om)
        ref = sum(2 * lam[k] / (lam[k] ** 2 + om ** 2) * np.vdot(U[:, k], rhs) * U[:, k] for k in cond)
        assert _rel(f, ref) < 1e-11


def test_gamma_basis_is_orthonormal_and_spans_its_input():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((5, 40)) + 1j * rng.standard_normal((5, 40))
    X = np.vstack([X, 0.3 * X[0] - 2j * X[2]])          # a dependent row is dropped
    G = gamma_basis(X)
    assert G.shape == (5, 40)
    assert np.abs(G.conj() @ G.T - np.eye(5)).max() < 1e-13
    assert np.abs(X - (X @ G.conj().T) @ G).max() < 1e-12


def test_finite_frequency_solution_improves_the_basis(c1):
    """Sec. VI's accuracy check: adding the solutions at w0 to the basis changes
    the result little, and moves it towards the direct projection at w0."""
    _, _, mf, Q = c1
    w0 = 1.0
    E = olz.project(mf.M, Q, [1j * w0])[0]
    e_base = _rel(recycled_E(mf, Q, [w0])[0], E)
    e_more = _rel(recycled_E(mf, Q, [w0], extra_w=(w0,))[0], E)
    print(f"recycled E(i): basis x(0), x(inf) {e_base:.2e}; with x(i) {e_more:.2e}")
    assert e_base < 5e-2
    assert e_more < e_base
