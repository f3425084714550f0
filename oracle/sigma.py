"""Correlation self-energy of Secs. II, III.B, IV and VI in the dielectric
basis: the integrand traces, the Lorentzian-model terms and the residues.

Test infrastructure (the oracle): used by tests/ only.

Notation.  e is the state being corrected and delta the energy offset of the
self-energy argument, s = eps_e + delta, omega_ne = eps_n - s.  The pair
function |n* e> is the grid function conj(phi_n) phi_e; v^1/2 is the
truncated Coulomb square root; a matrix element <f| A |g> of an operator
with grid matrix A (kernel times dV) is dV f^H A g.  The basis {l} is given
as k orthonormal grid vectors q_l (Euclidean norm), and eps^-1 - 1 enters
through the inverse taken within span(Q), Sec. IV:

    W(z) = (I + E(z))^-1 - I,   E(z) = Q^H (eps(z) - 1) Q.

Sum-over-states forms (Sec. II, Eqs. (dge), (dg0e), (dhe); every eigenstate
n of the dense H):

    sigma_N(i w)  = sum_n <en*| v^1/2 Q W(i w) Q^H v^1/2 |n*e> omega_ne / (w^2 + omega_ne^2)
    sigma_N0(i w) = f(w) sum_n <en*| v^1/2 Q W(0) Q^H v^1/2 |n*e> omega_ne / (w^2 + omega_ne^2)
    Sigma_A       = sum_n <en*| v^1/2 Q W(0) Q^H v^1/2 |n*e> F_ne

with the Lorentzian model f(w) = a^2 / (w^2 + a^2) of Sec. III.B and
F_ne = (1/pi) int_0^inf f(w) omega_ne / (w^2 + omega_ne^2) dw.

Trace forms (Sec. IV, Eq. (traces)): the same three numbers as traces over the
basis, with H inverted by linear solves instead of summed over eigenstates,

    sigma_N(i w) = Tr[W(i w) K(i w)],  K_{l'l} = (1/dV) g_l'^H (H - s)((H - s)^2 + w^2)^-1 g_l,
    g_l = Gather(conj(phi_e) v^1/2 q_l),

and Sigma_A with F_A(H) = (a/2) [Q_e (H - s + a)^-1 Q_e + P_e (H - s - a)^-1 P_e]
(Eqs. (he), (khe)); P_e projects on the states below s, Q_e on those above.

Residues (Eq. (pe), Sec. VI): for every valence state v with omega_ve > 0
(and conduction state c with omega_ce < 0), the matrix element
<ev*| v^1/2 (eps^-1(omega) - 1) v^1/2 |v*e> at the real frequency omega_ve,
from a Lanczos recursion on eps(omega) - 1 seeded with v^1/2 |v*e>:
|p|^2 [(I + T)^-1 - I]_00 dV.  Theta(0) = 1/2 (Eq. (theta)).

Readings (the paper's text is garbled or silent on these):
* F_ne for the Lorentzian model is (1/2) a / (omega_ne + a sgn(omega_ne));
  the printed prefactor pi/2 contradicts the definition (Fne) and the
  (1/2)-weighted Sigma_A of Eq. (he), both of which give 1/2.
* H* = H for a real local potential, so the conjugated operators of Eq.
  (traces) are H itself, and P_e*, Q_e* are H's spectral projectors.
* The frequency integral of Eq. (e_c) is the caller's quadrature; the
  footnote's map w = (1 + t) / (1 - t) with Gauss-Legendre nodes is given by
  gl_frequencies.
"""
from __future__ import annotations

import numpy as np

from .lanczos import lanczos
from .pw import Basis


def theta(x: float, atol: float = 1e-12) -> float:
    """Step function with Theta(0) = 1/2 (Eq. (theta))."""
    return 1.0 if x > atol else (0.5 if x >= -atol else 0.0)


def lorentz_f(w, alpha: float):
    """Model function f(w) = a^2 / (w^2 + a^2) of Sec. III.B."""
    return alpha ** 2 / (np.asarray(w, dtype=float) ** 2 + alpha ** 2)


def lorentz_F(wne, alpha: float, atol: float = 1e-12):
    """F_ne = (1/pi) int_0^inf f(w) wne / (w^2 + wne^2) dw for the Lorentzian:
    (1/2) a / (wne + a sgn(wne)); 0 when wne = 0 (half the pole on each side)."""
    wne = np.asarray(wne, dtype=float)
    sg = np.where(wne > atol, 1.0, np.where(wne < -atol, -1.0, 0.0))
    den = np.where(sg == 0.0, 1.0, wne + alpha * sg)
    return np.where(sg == 0.0, 0.0, 0.5 * alpha / den)


def gl_frequencies(n: int):
    """Gauss-Legendre nodes on (-1, 1) mapped by w = (1 + t) / (1 - t) to
    (0, inf): returns (w [n], weights [n]) with sum weights g(w) ~ int_0^inf g."""
    t, wt = np.polynomial.legendre.leggauss(n)
    return (1.0 + t) / (1.0 - t), wt * 2.0 / (1.0 - t) ** 2


def basis_W(E: np.ndarray) -> np.ndarray:
    """(I + E)^-1 - I for one k x k matrix E."""
    k = E.shape[0]
    return np.linalg.inv(np.eye(k) + E) - np.eye(k)


def project_E(apply_Mz, Q: np.ndarray, z: complex) -> np.ndarray:
    """E(z) = Q^H (eps(z) - 1) Q."""
    W = np.array([apply_Mz(z, q) for q in Q])
    return Q.conj() @ W.T


class SigmaSOS:
    """The sum-over-states forms over every eigenstate of the dense H.

    sos: an oracle.sos.SOS (all eigenpairs of the plane-wave H).  e: index of
    the corrected state in that spectrum.
    """

    def __init__(self, sos, e: int, delta: float, alpha: float = 1.0):
        self.sos, self.b = sos, sos.b
        self.e, self.delta, self.alpha = e, float(delta), float(alpha)
        self.s = sos.eps[e] + self.delta
        self.wne = sos.eps - self.s
        # v^1/2 |n* e> for every n: [N_pw, N^3]
        self.p = self.b.apply_vhalf(sos.psi.conj() * sos.psi[e][None, :])

    def _elements(self, Q: np.ndarray, W: np.ndarray) -> np.ndarray:
        """<en*| v^1/2 Q W Q^H v^1/2 |n*e> for every n."""
        A = Q.conj() @ self.p.T                       # [k, N_pw]: a_n = Q^H p_n
        return self.b.dV * np.sum(A.conj() * (W @ A), axis=0)

    def sigma_N(self, Q, W_iw, w: float) -> float:
        m = self._elements(Q, W_iw)
        return float(np.real(np.sum(m * self.wne / (w * w + self.wne ** 2))))

    def sigma_N0(self, Q, W0, w: float) -> float:
        m = self._elements(Q, W0)
        return float(lorentz_f(w, self.alpha) * np.real(np.sum(m * self.wne / (w * w + self.wne ** 2))))

    def sigma_A(self, Q, W0) -> float:
        m = self._elements(Q, W0)
        return float(np.real(np.sum(m * lorentz_F(self.wne, self.alpha))))

    def residue_element(self, n: int, omega: float, k: int | None = None) -> float:
        """<en*| v^1/2 (eps^-1(omega) - 1) v^1/2 |n*e> at real omega: by a k-step
        Lanczos recursion on eps(omega) - 1 seeded with v^1/2 |n*e> (Sec. VI),
        or with the dense inverse when k is None."""
        p = self.p[n]
        z = complex(omega, 0.0)
        if k is None:
            M = self.sos.M_matrix(z)
            n3 = M.shape[0]
            X = np.linalg.inv(np.eye(n3) + M) - np.eye(n3)
            return float(np.real(self.b.dV * np.vdot(p, X @ p)))
        a, bt, _, kd = lanczos(lambda v: self.sos.M(z, v), p, k)
        T = np.diag(a) + np.diag(bt[:kd - 1], 1) + np.diag(bt[:kd - 1], -1)
        X = np.linalg.inv(np.eye(kd) + T) - np.eye(kd)
        return float(self.b.dV * np.vdot(p, p).real * X[0, 0])

    def poles(self):
        """(n, weight, sign) of the residue terms: valence states with
        omega_ne > 0 enter with -Theta(omega_ne), conduction states with
        omega_ne < 0 with +Theta(-omega_ne)."""
        out = []
        for n, w in enumerate(self.wne):
            if n < self.sos.n_v:
                th = theta(w)
                if th > 0:
                    out.append((n, th, -1.0))
            else:
                th = theta(-w)
                if th > 0:
                    out.append((n, th, +1.0))
        return out

    def sigma_P(self, k: int | None = None) -> float:
        """Residue term Sigma_P of Eq. (pe)."""
        tot = 0.0
        for n, th, sg in self.poles():
            tot += sg * th * self.residue_element(n, float(self.wne[n]), k)
        return tot


class SigmaTrace:
    """The trace forms of Eq. (traces): H inverted by dense linear solves on
    the plane-wave sphere, no eigenvectors.

    psi_v, eps_v: the valence orbitals on the grid and their energies (the
    projectors P_e, Q_e of Eq. (khe) are built from them; s must lie below
    every conduction state).
    """

    def __init__(self, basis: Basis, V, psi_v, eps_v, e: int, delta: float, alpha: float = 1.0):
        self.b = basis
        H = basis.dense_H(V)
        self.H = 0.5 * (H + H.conj().T)
        self.psi_v = np.asarray(psi_v)
        self.eps_v = np.asarray(eps_v, dtype=float)
        self.e, self.delta, self.alpha = e, float(delta), float(alpha)
        self.s = self.eps_v[e] + self.delta
        self.U = basis.gather(self.psi_v.conj())     # [n_v, npw] sphere rows of conj(psi_v)

    def rhs(self, Q: np.ndarray) -> np.ndarray:
        """g_l = Gather(conj(phi_e) v^1/2 q_l): [k, npw]."""
        return self.b.gather(self.psi_v[self.e].conj()[None, :] * self.b.apply_vhalf(Q))

    def K(self, Q: np.ndarray, w: float) -> np.ndarray:
        """K(i w) = (1/dV) G^H (H - s)((H - s)^2 + w^2)^-1 G."""
        G = self.rhs(Q).T                              # [npw, k]
        A = self.H - self.s * np.eye(self.b.npw)
        Y = A @ np.linalg.solve(A @ A + (w * w) * np.eye(self.b.npw), G)
        return G.conj().T @ Y / self.b.dV

    def K_A(self, Q: np.ndarray) -> np.ndarray:
        """(1/dV) G^H F_A(H) G with F_A(H) = (a/2)[Q_e (H - s + a)^-1 Q_e + P_e (H - s - a)^-1 P_e]."""
        G = self.rhs(Q).T
        a = self.alpha
        th = np.array([theta(self.s - ev) for ev in self.eps_v])   # weight of P_e per band
        Pg = (self.U.T * (th == 1.0)[None, :]) @ self.U.conj()      # strictly below s
        Pq = np.eye(self.b.npw) - (self.U.T * (th > 0)[None, :]) @ self.U.conj()   # strictly above s
        I = np.eye(self.b.npw)
        A = self.H - self.s * I
        # Q_e part: solve on the range of Pq (the complement is made harmless by Pq)
        Yq = Pq @ np.linalg.solve(Pq @ (A + a * I) @ Pq + (I - Pq), Pq @ G)
        Yp = Pg @ np.linalg.solve(Pg @ (A - a * I) @ Pg + (I - Pg), Pg @ G)
        return 0.5 * a * (G.conj().T @ (Yq + Yp)) / self.b.dV

    def sigma_N(self, Q, W_iw, w: float) -> float:
        return float(np.real(np.trace(W_iw @ self.K(Q, w))))

    def sigma_N0(self, Q, W0, w: float) -> float:
        return float(lorentz_f(w, self.alpha) * np.real(np.trace(W0 @ self.K(Q, w))))

    def sigma_A(self, Q, W0) -> float:
        return float(np.real(np.trace(W0 @ self.K_A(Q))))
