"""Frequency recycling of Sec. VI: one small basis per valence band.

Test infrastructure (the oracle): used by tests/, smoke() and the CPU
baseline of bench.py only.

Sec. VI reuses the work of the static dielectric matrix at every imaginary
frequency.  For each valence band v, the static basis vectors l give
right-hand sides b_{l,v} = P_c* Gather(conj psi_v v^1/2 q_l) (Eq. (recy_eq));
their solutions at zero frequency x_{l,v}(0), already computed for eps(0),
and the large-frequency directions (H - e_v) b_{l,v} (the limit of the
solution times w^2) are turned into an orthonormal basis {gamma_{i,v}} by a
singular value decomposition.  H - e_v and the right-hand sides are expressed
in that basis once, and the imaginary-axis equation is solved in it by direct
inversion at every frequency.

Reading used here (the paper names the ingredients, not the small-matrix
formula): with h_v = gamma^H (H - e_v) gamma, the imaginary-axis solution
f = 2 (H - e_v) ((H - e_v)^2 + w^2)^-1 b of Sec. III.A is approximated by

    f ~ gamma  2 h_v (h_v^2 + w^2)^-1  gamma^H b,

the same function of the projected operator.  It is exact at w = 0 (x(0) lies
in the basis, and h_v is the Galerkin matrix of H - e_v), and exact at every
w when the basis is an invariant subspace of P(H - e_v)P containing b.
Columns whose singular value is below rtol times the largest are dropped.
"""
from __future__ import annotations

import numpy as np

from .sternheimer import MatrixFree


def gamma_basis(vectors: np.ndarray, rtol: float = 1e-10) -> np.ndarray:
    """Orthonormal rows spanning the rows of `vectors` [n, npw] (SVD, Sec. VI);
    directions with singular value below rtol * max are dropped."""
    U, s, _ = np.linalg.svd(np.asarray(vectors).T, full_matrices=False)
    keep = s > rtol * s[0]
    return U[:, keep].T.copy()


def projected_h(mf: MatrixFree, v: int, G: np.ndarray) -> np.ndarray:
    """h = G^H (P (H - e_v) P) G for basis rows G, made exactly Hermitian."""
    e = mf.eps_v[v]
    HG = np.array([mf.P(mf.H(mf.P(g)) - e * mf.P(g)) for g in G])
    h = G.conj() @ HG.T
    return 0.5 * (h + h.conj().T)


def solve_in_basis(h: np.ndarray, bg: np.ndarray, w: float) -> np.ndarray:
    """Coefficients c = 2 h (h^2 + w^2)^-1 bg (bg: [r] or [r, m])."""
    r = h.shape[0]
    return 2.0 * h @ np.linalg.solve(h @ h + (w * w) * np.eye(r), bg)


def band_rhs(mf: MatrixFree, xg: np.ndarray) -> np.ndarray:
    """b_{l,v} = P Gather(conj psi_v x) for all bands v: [n_v, npw]."""
    return np.array([mf.P(mf.b.gather(mf.psi_v[v].conj() * xg)) for v in range(len(mf.eps_v))])


def recycle_bases(mf: MatrixFree, Q: np.ndarray, rtol: float = 1e-10, extra_w=()):
    """Per band: the basis rows G_v from {x_{l,v}(0)} and {P (H - e_v) b_{l,v}}
    over the static basis Q [k, N^3] (plus the solutions at the imaginary
    frequencies in extra_w, the accuracy check of Sec. VI), and the right-hand
    sides B_v [k, npw]."""
    nv = len(mf.eps_v)
    B = np.array([band_rhs(mf, mf.b.apply_vhalf(q)) for q in Q])        # [k, n_v, npw]
    bases = []
    for v in range(nv):
        e = mf.eps_v[v]
        vec = [mf.solve_band(v, 0.0, B[l, v]) for l in range(len(Q))]
        vec += [mf.P(mf.H(B[l, v]) - e * B[l, v]) for l in range(len(Q))]
        for w in extra_w:
            vec += [mf.solve_band(v, 1j * w, B[l, v]) for l in range(len(Q))]
        bases.append(gamma_basis(np.array(vec), rtol))
    return bases, B


def recycled_E(mf: MatrixFree, Q: np.ndarray, w_list, bases=None, rtol: float = 1e-10, extra_w=()):
    """E(i w) = Q^H (eps(i w) - 1) Q for each w in w_list [n_w, k, k], with
    every band solve done in its recycled basis (given, or built from Q)."""
    if bases is None:
        bases, B = recycle_bases(mf, Q, rtol, extra_w)
    else:
        B = np.array([band_rhs(mf, mf.b.apply_vhalf(q)) for q in Q])
    nv = len(mf.eps_v)
    hs = [projected_h(mf, v, bases[v]) for v in range(nv)]
    out = []
    for w in w_list:
        W = []
        for l in range(len(Q)):
            chi = np.zeros(mf.b.N ** 3, dtype=np.complex128)
            for v in range(nv):
                G = bases[v]
                c = solve_in_basis(hs[v], G.conj() @ B[l, v], float(w))
                f = G.T @ c
                chi += -2.0 * mf.psi_v[v] * mf.b.scatter(f)
            W.append(-mf.b.apply_vhalf(chi))
        out.append(Q.conj() @ np.array(W).T)
    return np.array(out)
