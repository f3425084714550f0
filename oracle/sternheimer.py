"""chi0 through the Sternheimer equations of Sec. III.A.

Completeness, sum_c |c><c| = 1 - sum_v |v><v| = P_c, turns the sum over
conduction states of Sec. II into linear systems, one per valence band:

    (H - e_v -+ z) f_-+ = P_c* b_v,   b_v = Gather(conj(psi_v) x),
    chi0(z) x = -2 sum_v psi_v Scatter(f_- + f_+).

The projector acts on the conjugated valence set because the pair function of
Sec. II pairs conj(psi_c) with psi_v; for a real local potential H* = H as an
operator on grid functions, so the systems use H itself (the reading of the
recycling formula of Sec. VI).  On the imaginary axis z = i w the two systems
combine into the Hermitian positive-definite equation of Sec. III.A,

    ((H - e_v)^2 + w^2) f = 2 (H - e_v) P_c* b_v,   f = f_+ + f_-,

and at w = 0 into (H - e_v) f = 2 P_c* b_v on the conduction subspace, made
non-singular by projecting out the valence subspace (Sec. III.A).

``dense_chi0`` solves these equations with dense LU (the O1 cross-check of
completeness); ``MatrixFree`` solves them with SciPy Krylov solvers on
FFT-applied H (O2, for grids too large to diagonalise).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .pw import Basis


def _valence_conj(basis: Basis, psi_v: np.ndarray) -> np.ndarray:
    """Sphere coefficients of conj(psi_v), orthonormalised (QR) for the projector."""
    U = basis.gather(psi_v.conj())                    # [n_v, npw]
    Q, _ = np.linalg.qr(U.T)
    return Q.T.copy()


def dense_chi0(basis: Basis, V, psi_v, eps_v, z: complex, x: np.ndarray) -> np.ndarray:
    """chi0(z) x with each Sternheimer system solved densely (numpy LU).

    The valence block is made non-singular with the beta P_v shift of
    Sec. III.A (beta = 1 here); the right-hand side has no valence component
    so the shift does not change the solution.
    """
    H = basis.dense_H(V)
    H = 0.5 * (H + H.conj().T)
    U = _valence_conj(basis, psi_v)
    Pv = U.T @ U.conj()                                # projector on span{conj(psi_v)}
    Pc = np.eye(basis.npw) - Pv
    I = np.eye(basis.npw)
    out = np.zeros(basis.N ** 3, dtype=np.complex128)
    for v in range(len(eps_v)):
        b = Pc @ basis.gather(psi_v[v].conj() * x)
        A = H - eps_v[v] * I
        if z.real == 0.0:
            w = z.imag
            lhs = Pc @ (A @ A + w * w * I) @ Pc + Pv
            f = np.linalg.solve(lhs, 2.0 * (Pc @ (A @ b)))
        else:
            fm = np.linalg.solve(Pc @ (A - z * I) @ Pc + Pv, b)
            fp = np.linalg.solve(Pc @ (A + z * I) @ Pc + Pv, b)
            f = fm + fp
        out += -2.0 * psi_v[v] * basis.scatter(f)
    return out


class MatrixFree:
    """O2: matrix-free FP64 Sternheimer chi0 with SciPy Krylov solvers.

    Imaginary axis (including 0): conjugate gradients on the Hermitian
    positive-definite projected system.  Real axis with broadening:
    restarted GMRES on each of the two shifted systems (a different Krylov
    method from the SQMR of the HIP library, on purpose).
    """

    def __init__(self, basis: Basis, V, psi_v, eps_v, rtol: float = 1e-13,
                 maxiter: int = 20000):
        self.b = basis
        self.V = np.asarray(V, dtype=np.float64).reshape(-1)
        self.psi_v = np.asarray(psi_v)
        self.eps_v = np.asarray(eps_v, dtype=np.float64)
        self.U = _valence_conj(basis, self.psi_v)
        self.rtol, self.maxiter = rtol, maxiter
        self.iters: list[int] = []

    def P(self, c):
        return c - self.U.T @ (self.U.conj() @ c)

    def H(self, c):
        return self.b.apply_H(self.V, c)

    def _solve_hpd(self, op, rhs):
        n = self.b.npw
        A = spla.LinearOperator((n, n), matvec=op, dtype=np.complex128)
        count = [0]

        def cb(_):
            count[0] += 1
        f, info = spla.cg(A, rhs, rtol=self.rtol, atol=0.0, maxiter=self.maxiter,
                          callback=cb)
        self.iters.append(count[0])
        if info != 0:
            raise RuntimeError(f"oracle CG did not converge (info={info})")
        return f

    def _solve_gen(self, op, rhs):
        n = self.b.npw
        A = spla.LinearOperator((n, n), matvec=op, dtype=np.complex128)
        count = [0]

        def cb(_):
            count[0] += 1
        f, info = spla.gmres(A, rhs, rtol=self.rtol, atol=0.0, restart=400,
                             maxiter=self.maxiter, callback=cb, callback_type="pr_norm")
        self.iters.append(count[0])
        if info != 0:
            raise RuntimeError(f"oracle GMRES did not converge (info={info})")
        return f

    def solve_band(self, v: int, z: complex, b: np.ndarray) -> np.ndarray:
        """f = f_- + f_+ for band v (b already projected)."""
        e = self.eps_v[v]
        if z.real == 0.0:
            w2 = z.imag ** 2
            if w2 == 0.0:
                return 2.0 * self._solve_hpd(lambda c: self.P(self.H(self.P(c)) - e * self.P(c)), b)
            rhs = 2.0 * self.P(self.H(b) - e * b)

            def op(c):
                c = self.P(c)
                a = self.H(c) - e * c
                return self.P(self.H(a) - e * a + w2 * c)
            return self._solve_hpd(op, rhs)
        fm = self._solve_gen(lambda c: self.P(self.H(self.P(c)) - (e + z) * self.P(c)), b)
        fp = self._solve_gen(lambda c: self.P(self.H(self.P(c)) - (e - z) * self.P(c)), b)
        return fm + fp

    def chi0(self, z: complex, x: np.ndarray) -> np.ndarray:
        """chi0(z) x for one grid vector x [N^3]."""
        out = np.zeros(self.b.N ** 3, dtype=np.complex128)
        for v in range(len(self.eps_v)):
            b = self.P(self.b.gather(self.psi_v[v].conj() * x))
            f = self.solve_band(v, complex(z), b)
            out += -2.0 * self.psi_v[v] * self.b.scatter(f)
        return out

    def M(self, z: complex, x: np.ndarray) -> np.ndarray:
        """eps(z) - 1 = -v^(1/2) chi0(z) v^(1/2) x."""
        return -self.b.apply_vhalf(self.chi0(z, self.b.apply_vhalf(x)))
