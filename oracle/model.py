"""The model dielectric operator of Sec. V (Eq. (model_eq)): H -> T.

Test infrastructure (the oracle): used by tests/, smoke() and the CPU
baseline of bench.py only.

Sec. V replaces the Hamiltonian by the kinetic operator T (diagonal in plane
waves) in the Sternheimer equations, so that each band's solution is one
diagonal division between two conduction projections instead of a Krylov
solve:

    f~_{v,-+} = P_c (T - e_v -+ z)^-1 P_c b_v,   b_v = P_c Gather(conj psi_v x),
    chi0~(z) x = -2 sum_v psi_v Scatter(f~_- + f~_+),
    eps~(z) - 1 = -v^1/2 chi0~(z) v^1/2,

in the same conjugation reading as the exact operator (oracle/sternheimer.py);
a term whose denominator vanishes is dropped.
With V_loc = 0 the valence states are plane waves, T commutes with P_c and the
model is exact (the Lindhard closed form).
"""
from __future__ import annotations

import numpy as np

from .pw import Basis
from .sternheimer import _valence_conj


def _div(b, d):
    """b / d with the terms of vanishing denominator dropped (in the free box
    they fall on valence plane waves, where the projected b is zero)."""
    out = np.zeros_like(b)
    nz = d != 0
    out[nz] = b[nz] / d[nz]
    return out


class Model:
    def __init__(self, basis: Basis, psi_v, eps_v):
        self.b = basis
        self.psi_v = np.asarray(psi_v)
        self.eps_v = np.asarray(eps_v, dtype=np.float64)
        self.U = _valence_conj(basis, self.psi_v)

    def P(self, c):
        return c - self.U.T @ (self.U.conj() @ c)

    def chi0(self, z: complex, x: np.ndarray) -> np.ndarray:
        """chi0~(z) x for one grid vector x [N^3]."""
        z = complex(z)
        out = np.zeros(self.b.N ** 3, dtype=np.complex128)
        for v in range(len(self.eps_v)):
            bv = self.P(self.b.gather(self.psi_v[v].conj() * x))
            d = self.b.kin - self.eps_v[v]
            f = self.P(_div(bv, d - z) + _div(bv, d + z))
            out += -2.0 * self.psi_v[v] * self.b.scatter(f)
        return out

    def M(self, z: complex, x: np.ndarray) -> np.ndarray:
        """eps~(z) - 1 = -v^(1/2) chi0~(z) v^(1/2) x."""
        return -self.b.apply_vhalf(self.chi0(z, self.b.apply_vhalf(x)))
