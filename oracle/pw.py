"""Discrete plane-wave problem (oracle side).

The paper works in ABINIT's plane-wave representation without spelling out the
discretisation (Sec. IX uses a cubic cell, a kinetic cut-off and a spherical
Coulomb truncation).  The reading used here:

* grid r_n = L n / N, n in {0..N-1}^3, volume Omega = L^3, dV = Omega / N^3;
* reciprocal vectors K_m = 2 pi m / L with m the signed FFT integers;
* sphere S = {m : |K_m|^2 / 2 <= ecut};
* an orbital with sphere coefficients c is psi(r_n) = Omega^(-1/2) sum_m c_m e^{i K_m r_n},
  so that dV sum_n conj(f) g = c^H d for orbitals;
* Gather(g)_m = Omega^(1/2) N^-3 sum_n g(r_n) e^{-i K_m r_n}   (grid -> sphere);
* Scatter(y)(r_n) = Omega^(-1/2) sum_m y_m e^{i K_m r_n}       (sphere -> grid);
* H = |K|^2/2 + V_loc, with the potential applied on the grid (circular
  convolution in the sphere basis).
"""
from __future__ import annotations

import numpy as np


class Basis:
    """Grid and plane-wave sphere of a cubic box (oracle's own enumeration)."""

    def __init__(self, L: float, N: int, ecut: float):
        self.L, self.N, self.ecut = float(L), int(N), float(ecut)
        self.omega = self.L ** 3
        self.dV = self.omega / self.N ** 3
        f = np.fft.fftfreq(N, d=1.0 / N).astype(np.int64)   # signed integers
        self.freq = f
        mx, my, mz = np.meshgrid(f, f, f, indexing="ij")
        self.k2_grid = (2 * np.pi / L) ** 2 * (mx ** 2 + my ** 2 + mz ** 2)
        sel = (0.5 * self.k2_grid <= ecut).ravel()
        self.idx = np.flatnonzero(sel)                       # flat grid index of each PW
        self.m = np.stack([mx.ravel()[self.idx], my.ravel()[self.idx],
                           mz.ravel()[self.idx]], axis=1)
        if np.abs(self.m).max() > N // 2 - 1:
            raise ValueError("plane-wave sphere does not fit in the grid")
        self.kin = 0.5 * self.k2_grid.ravel()[self.idx]
        self.npw = self.idx.size

    # --- transforms -------------------------------------------------------
    def gather(self, g: np.ndarray) -> np.ndarray:
        """Grid function(s) [..., N^3] -> sphere coefficients [..., npw]."""
        N = self.N
        g = np.asarray(g).reshape(g.shape[:-1] + (N, N, N))
        G = np.fft.fftn(g, axes=(-3, -2, -1)).reshape(g.shape[:-3] + (N ** 3,))
        return G[..., self.idx] * (np.sqrt(self.omega) / N ** 3)

    def scatter(self, y: np.ndarray) -> np.ndarray:
        """Sphere coefficients [..., npw] -> grid function(s) [..., N^3]."""
        N = self.N
        y = np.asarray(y)
        G = np.zeros(y.shape[:-1] + (N ** 3,), dtype=np.complex128)
        G[..., self.idx] = y
        G = G.reshape(y.shape[:-1] + (N, N, N))
        g = np.fft.ifftn(G, axes=(-3, -2, -1)) * (N ** 3 / np.sqrt(self.omega))
        return g.reshape(y.shape[:-1] + (N ** 3,))

    # --- Hamiltonian ------------------------------------------------------
    def dense_H(self, V: np.ndarray) -> np.ndarray:
        """Dense H_{ab} = kin_a delta_ab + Vhat((m_a - m_b) mod N), Vhat = FFT(V)/N^3."""
        N = self.N
        Vg = np.fft.fftn(np.asarray(V, dtype=np.float64).reshape(N, N, N)) / N ** 3
        d = (self.m[:, None, :] - self.m[None, :, :]) % N
        H = Vg[d[..., 0], d[..., 1], d[..., 2]].astype(np.complex128)
        H[np.diag_indices(self.npw)] += self.kin
        return H

    def apply_H(self, V: np.ndarray, c: np.ndarray) -> np.ndarray:
        """Matrix-free H c = kin c + Gather(V * Scatter(c)) for c [..., npw]."""
        Vr = np.asarray(V, dtype=np.float64).reshape(-1)
        return self.kin * c + self.gather(Vr * self.scatter(c))

    # --- Coulomb ----------------------------------------------------------
    def sqrt_coulomb(self) -> np.ndarray:
        """sqrt(v(K)) on the full grid for the spherically truncated Coulomb kernel.

        Sec. IX truncates 1/r at a radius of half the cubic cell.  The Fourier
        transform of 1/r restricted to r < R is 4 pi (1 - cos(K R)) / K^2, with
        the limit 2 pi R^2 at K = 0.
        """
        R = self.L / 2
        k2 = self.k2_grid.ravel()
        k = np.sqrt(k2)
        v = np.empty_like(k2)
        nz = k2 > 0
        v[nz] = 4 * np.pi * (1 - np.cos(k[nz] * R)) / k2[nz]
        v[~nz] = 2 * np.pi * R ** 2
        return np.sqrt(v)

    def apply_vhalf(self, x: np.ndarray) -> np.ndarray:
        """v^(1/2) x = IFFT(sqrt(v(K)) FFT(x)) over the full grid, x [..., N^3]."""
        N = self.N
        s = self.sqrt_coulomb().reshape(N, N, N)
        X = np.asarray(x).reshape(x.shape[:-1] + (N, N, N))
        y = np.fft.ifftn(s * np.fft.fftn(X, axes=(-3, -2, -1)), axes=(-3, -2, -1))
        return y.reshape(x.shape)
