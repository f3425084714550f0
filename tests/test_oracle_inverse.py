"""Pins of the oracle's inverse in the Lanczos basis and its Ritz values
(Sec. IV) against what the mathematics fixes: on an invariant subspace of
eps(z) the basis inverse is eps(z)^-1 itself (checked by a dense linear solve
of eps y = x), a full Lanczos recursion's Ritz values are the spectrum, and
Ritz values of successive steps interlace."""
import numpy as np

from oracle import lanczos as olz
from oracle.pw import Basis
from oracle.sos import SOS
from synthetic import gaussian_wells, random_potentials
from synthetic.ground_state import ground_state


def _small_box():
    L, N, ecut, n_v = 6.0, 8, 4.0, 2
    V = gaussian_wells(L, N, 2, np.random.default_rng([14083036, 99, 1]))
    psi, eps, _ = ground_state(V, L, ecut, n_v)
    b = Basis(L, N, ecut)
    return b, SOS(b, V, n_v)


def test_basis_inverse_on_an_invariant_subspace_is_eps_inverse():
    b, s = _small_box()
    for z in (0.0, 0.7j):
        M = s.M_matrix(z)                         # eps(z) - 1, Hermitian on the imaginary axis
        lam, U = np.linalg.eigh(0.5 * (M + M.conj().T))
        pick = [len(lam) - 1, len(lam) - 2, len(lam) - 5, len(lam) // 2]
        Q = U[:, pick].T                          # rows: an orthonormal invariant basis
        E = Q.conj() @ (M @ Q.T)
        Einv = olz.eps_inverse_in_basis(E[None])[0]
        rng = np.random.default_rng(5)
        x = Q.T @ (rng.standard_normal(len(pick)) + 1j * rng.standard_normal(len(pick)))
        y_dense = np.linalg.solve(np.eye(len(M)) + M, x)     # eps^-1 x
        y_basis = x + Q.T @ ((Einv - np.eye(len(pick))) @ (Q.conj() @ x))
        assert np.linalg.norm(y_basis - y_dense) < 1e-12 * np.linalg.norm(y_dense)
        # eigenvalues of the inverse: 1 / (1 + theta), and 1 - eps^-1 in [0, 1)
        mu = np.linalg.eigvalsh(0.5 * (Einv + Einv.conj().T))
        assert np.allclose(np.sort(mu), np.sort(1.0 / (1.0 + lam[pick])), rtol=1e-12, atol=1e-14)
        assert np.all(1.0 - mu >= -1e-14) and np.all(1.0 - mu < 1.0)


def test_ritz_values_of_a_full_recursion_are_the_spectrum():
    rng = np.random.default_rng(11)
    n = 24
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    M = A @ A.conj().T / n                        # Hermitian positive semidefinite
    q0 = rng.standard_normal(n)
    a, be, Q, kd = olz.lanczos(lambda v: M @ v, q0, n)
    th = olz.ritz_values(a[:kd], be[:kd])
    lam = np.linalg.eigvalsh(M)
    assert kd == n
    assert np.abs(th - lam).max() < 1e-10 * lam.max()


def test_ritz_values_interlace_and_stay_in_the_spectrum():
    b, s = _small_box()
    M = s.M_matrix(0.0)
    lam = np.linalg.eigvalsh(0.5 * (M + M.conj().T))
    q0 = random_potentials(b.N, 1, 12)[0]
    a, be, Q, kd = olz.lanczos(lambda v: M @ v, q0, 10)
    prev = None
    for k in range(1, kd + 1):
        th = olz.ritz_values(a[:k], be[:k])
        assert th.min() >= lam.min() - 1e-12 and th.max() <= lam.max() + 1e-12
        if prev is not None:                      # Cauchy interlacing of T_k and T_{k-1}
            assert np.all(th[:-1] <= prev + 1e-12) and np.all(prev <= th[1:] + 1e-12)
        prev = th
