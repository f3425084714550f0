"""Pins of the model dielectric operator oracle (Sec. V, oracle/model.py):
the Lindhard closed form at V_loc = 0, where H = T and the model is exact, and
Hermiticity and sign of chi0~ on the imaginary axis with a potential."""
import numpy as np
import pytest

from oracle import lindhard
from oracle.model import Model
from oracle.pw import Basis
from synthetic import make_workload

L1, N1, E1 = 10.0, 16, 6.0


def _plane_wave(L, N, q):
    r = L * np.stack(np.meshgrid(*[np.arange(N)] * 3, indexing="ij"), -1).reshape(-1, 3) / N
    return np.exp(1j * (2 * np.pi / L) * r @ np.asarray(q, float))


@pytest.mark.parametrize("n_v", [1, 7])
def test_model_is_lindhard_without_potential(n_v):
    """V_loc = 0: the valence states are the n_v lowest plane waves (a closed
    shell), and chi0~ has the closed-form eigenvalues of the free box."""
    b = Basis(L1, N1, E1)
    pts = lindhard.sphere_triples(L1, N1, E1)
    val, _ = lindhard.closed_shell_valence(pts, n_v)
    psi = np.array([_plane_wave(L1, N1, m) / np.sqrt(b.omega) for m, _ in val])
    eps = np.array([e for _, e in val])
    md = Model(b, psi, eps)
    for q in [(1, 0, 0), (2, 1, 0), (3, -2, 1), (7, 7, 7)]:
        x = _plane_wave(L1, N1, q)
        for z in [0.0, 0.3j, 0.5 + 0.01j, -0.2 + 0.003j]:
            lam = lindhard.eigenvalue(L1, N1, E1, n_v, q, z)
            y = md.chi0(z, x)
            assert np.abs(y - lam * x).max() <= 1e-12 * max(abs(lam), 1e-2)


def test_model_hermitian_and_negative_on_imaginary_axis():
    """With a potential: chi0~(i w) is Hermitian and negative semidefinite
    (each band contributes -4 P D (D^2 + w^2)^-1 P with D = T - e_v > 0)."""
    w = make_workload(1, L=8.0, N=12, ecut=4.0)
    b = Basis(w.L, w.N, w.ecut)
    md = Model(b, w.psi, w.eps)
    assert np.all(w.eps < 0)
    n = w.N ** 3
    for om in (0.0, 0.6):
        X = np.array([md.chi0(1j * om, e) for e in np.eye(n)]).T
        assert np.abs(X - X.conj().T).max() < 1e-13 * np.abs(X).max()
        ev = np.linalg.eigvalsh(0.5 * (X + X.conj().T))
        assert ev.max() <= 1e-12 * np.abs(ev).max()
