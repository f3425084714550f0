"""O1: chi0 by the explicit sum over all conduction states (Sec. II).

The Adler-Wiser random-phase polarizability of Sec. II is, for a spin-
unpolarised molecule (factor 2),

    P(z) = 2 sum_{c,v} |c* v> [1/(z - (e_c - e_v)) - 1/(z + (e_c - e_v))] <v c*|,

where |c* v> is the grid function conj(psi_c) psi_v.  Here every eigenpair of
the dense plane-wave Hamiltonian is computed, the N_v lowest are the valence
set and all the others the conduction set, and the sum is carried out
literally.  On the imaginary axis the same sum is the negative semidefinite
operator written in Sec. VI (each term 4 (e_c-e_v)/((e_c-e_v)^2 + w^2)).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .pw import Basis


class SOS:
    """Dense eigen-decomposition of H and the explicit pair sum for chi0."""

    def __init__(self, basis: Basis, V: np.ndarray, n_v: int):
        self.b = basis
        self.n_v = n_v
        H = basis.dense_H(V)
        H = 0.5 * (H + H.conj().T)
        self.eps, self.C = scipy.linalg.eigh(H)          # all N_pw eigenpairs
        if self.eps[n_v] - self.eps[n_v - 1] < 1e-9:
            raise ValueError("valence set splits a degenerate level")
        self.psi = basis.scatter(self.C.T)                # [N_pw, N^3] grid orbitals
        psi_v = self.psi[:n_v]
        psi_c = self.psi[n_v:]
        # pair functions rho_cv(r) = conj(psi_c(r)) psi_v(r), ordered (v, c)
        self.rho = (psi_v[:, None, :] * psi_c.conj()[None, :, :]).reshape(-1, basis.N ** 3)
        self.delta = (self.eps[n_v:][None, :] - self.eps[:n_v][:, None]).reshape(-1)

    def weights(self, z: complex) -> np.ndarray:
        """2 [1/(z - D) - 1/(z + D)] for every (v, c) pair."""
        D = self.delta
        return 2.0 * (1.0 / (z - D) - 1.0 / (z + D))

    def chi0(self, z: complex, x: np.ndarray) -> np.ndarray:
        """chi0(z) x = sum_{cv} w_cv rho_cv <rho_cv, x>, <f,g> = dV sum conj(f) g.

        x: [..., N^3] complex.  Returns the same shape.
        """
        x2 = np.atleast_2d(x)
        proj = self.b.dV * (self.rho.conj() @ x2.T)       # [pairs, ncol]
        out = (self.rho.T @ (self.weights(z)[:, None] * proj)).T
        return out.reshape(np.shape(x))

    def chi0_matrix(self, z: complex) -> np.ndarray:
        """Dense chi0(z) as an N^3 x N^3 matrix acting on grid values."""
        w = self.weights(z)
        return self.b.dV * (self.rho.T * w[None, :]) @ self.rho.conj()

    def M(self, z: complex, x: np.ndarray) -> np.ndarray:
        """eps(z) - 1 = -v^(1/2) chi0(z) v^(1/2) applied to x (symmetrised form, Sec. II)."""
        return -self.b.apply_vhalf(self.chi0(z, self.b.apply_vhalf(x)))

    def M_matrix(self, z: complex) -> np.ndarray:
        """Dense eps(z) - 1 on the grid (N^3 x N^3)."""
        n3 = self.b.N ** 3
        X = self.chi0_matrix(z)
        # v^(1/2) X v^(1/2): apply on columns, then on rows (v^(1/2) is Hermitian)
        Y = self.b.apply_vhalf(X.T).T
        Y = self.b.apply_vhalf(Y)
        assert Y.shape == (n3, n3)
        return -Y
