"""Lowest eigenpairs of the model Hamiltonian, standing in for DFT valence states.

The plane-wave model: on the cubic box of edge L with an N^3 grid, orbitals are
expanded on the sphere S = {m : |2 pi m / L|^2 / 2 <= ecut} of signed integer
triples, psi(r_n) = Omega^(-1/2) sum_m c_m exp(i K_m . r_n), and the Hamiltonian
acts as kinetic |K|^2/2 plus the local potential applied on the grid.  This
module solves for the lowest eigenpairs only; it is input generation, written
independently of both the oracle and the HIP library (each of which checks the
eigen-residual of what it is given against its own Hamiltonian).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse.linalg as spla


def _sphere(L: float, N: int, ecut: float):
    f = np.fft.fftfreq(N, d=1.0 / N).astype(np.int64)
    mx, my, mz = np.meshgrid(f, f, f, indexing="ij")
    k2 = (2 * np.pi / L) ** 2 * (mx ** 2 + my ** 2 + mz ** 2)
    sel = 0.5 * k2 <= ecut
    idx = np.flatnonzero(sel.ravel())          # flat grid indices (x slowest)
    m = np.stack([mx.ravel()[idx], my.ravel()[idx], mz.ravel()[idx]], axis=1)
    if np.abs(m).max() > N // 2 - 1:
        raise ValueError("plane-wave sphere does not fit the grid")
    return idx, m, 0.5 * k2.ravel()[idx]


def ground_state(V: np.ndarray, L: float, ecut: float, n_v: int, n_extra: int = 4,
                 dense_limit: int = 4000):
    """Return (psi [n_v, N^3] complex128 grid orbitals, eps [n_v], eps_all [n_v+n_extra]).

    Orbitals are normalised so that dV * sum |psi|^2 = 1 (dV = L^3 / N^3).
    """
    N = V.shape[0]
    idx, m, kin = _sphere(L, N, ecut)
    npw = idx.size
    Vg = np.fft.fftn(V) / N ** 3
    nev = n_v + n_extra
    if npw <= dense_limit:
        # H_{ab} = kin_a delta_ab + Vhat((m_a - m_b) mod N)
        d = (m[:, None, :] - m[None, :, :]) % N
        H = Vg[d[..., 0], d[..., 1], d[..., 2]]
        H[np.diag_indices(npw)] += kin
        H = 0.5 * (H + H.conj().T)
        w, C = scipy.linalg.eigh(H, subset_by_index=[0, nev - 1])
    else:
        grid = np.zeros(N ** 3, dtype=np.complex128)

        def matvec(c):
            c = np.asarray(c).reshape(-1)
            grid[:] = 0
            grid[idx] = c
            g = np.fft.ifftn(grid.reshape(N, N, N)) * V
            return kin * c + np.fft.fftn(g).ravel()[idx]

        op = spla.LinearOperator((npw, npw), matvec=matvec, dtype=np.complex128)
        rng = np.random.default_rng(0)
        v0 = rng.standard_normal(npw) + 0j
        w, C = spla.eigsh(op, k=nev, which="SA", tol=1e-14, v0=v0,
                          ncv=max(4 * nev, 40), maxiter=100000)
        # Rayleigh-Ritz on the converged subspace: for a complex operator the
        # Krylov eigensolver's vectors within a degenerate level need not be
        # orthogonal; an orthonormal basis of the subspace and the eigenvectors
        # of H projected on it are
        C, _ = np.linalg.qr(C)
        HC = np.stack([matvec(C[:, i]) for i in range(nev)], axis=1)
        Hs = C.conj().T @ HC
        w, U = scipy.linalg.eigh(0.5 * (Hs + Hs.conj().T))
        C = C @ U
    C = C[:, :n_v]
    grid = np.zeros((n_v, N ** 3), dtype=np.complex128)
    grid[:, idx] = C.T
    omega = L ** 3
    psi = np.fft.ifftn(grid.reshape(n_v, N, N, N), axes=(1, 2, 3)).reshape(n_v, -1)
    psi *= N ** 3 / np.sqrt(omega)
    return psi, w[:n_v].copy(), w.copy()
