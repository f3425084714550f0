"""Lanczos basis of eps - 1 with full reorthogonalisation (Sec. IV), and the
projection of eps(z) - 1 on that static basis (Sec. VI).

Sec. IV builds the Krylov space {q, M q, M^2 q, ...} of the Hermitian positive
semidefinite operator M = eps(0) - 1 with the Lanczos procedure, so that M is
tridiagonal in the resulting orthonormal basis, and adds a Gram-Schmidt
orthogonalisation of every new residual against all previous Lanczos vectors.
The reading used here (Euclidean norm on grid values, classical Gram-Schmidt
applied twice):

    q_0 = q / |q|,  beta_0 = 0
    w = M q_j;  alpha_j = Re <q_j, w>;  w -= alpha_j q_j + beta_j q_{j-1}
    w -= Q (Q^H w)  (twice);  beta_{j+1} = |w|;  q_{j+1} = w / beta_{j+1}

It stops early on an invariant subspace (beta < 1e-14 max|alpha|).  Sec. VI
keeps this static basis for all imaginary frequencies; ``project`` returns
E(z) = Q^H (eps(z) - 1) Q.
"""
from __future__ import annotations

import numpy as np


def lanczos(apply_M, q0: np.ndarray, k: int, breakdown: float = 1e-14):
    """Return (alpha [k_done], beta [k_done], Q [k_done, n], k_done).

    beta[j] couples q_j and q_{j+1}; beta[k_done-1] is the final residual norm.
    """
    q = np.asarray(q0, dtype=np.complex128)
    q = q / np.linalg.norm(q)
    Q = [q]
    alpha, beta = [], []
    b_prev = 0.0
    for j in range(k):
        w = apply_M(Q[j])
        a = float(np.real(np.vdot(Q[j], w)))
        w = w - a * Q[j]
        if j > 0:
            w = w - b_prev * Q[j - 1]
        Qm = np.array(Q)
        for _ in range(2):
            w = w - Qm.T @ (Qm.conj() @ w)
        bnext = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(bnext)
        if bnext < breakdown * max(abs(x) for x in alpha):
            return np.array(alpha), np.array(beta), Qm, j + 1
        if j + 1 < k:
            Q.append(w / bnext)
        b_prev = bnext
    return np.array(alpha), np.array(beta), np.array(Q), k


def tridiag(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """Dense T with alpha on the diagonal and beta[:-1] on the off-diagonals."""
    k = len(alpha)
    T = np.diag(np.asarray(alpha, dtype=np.float64))
    if k > 1:
        T += np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)
    return T


def project(apply_Mz, Q: np.ndarray, z_list) -> np.ndarray:
    """E(z) = Q^H (eps(z) - 1) Q for each z: [n_z, k, k]."""
    out = []
    for z in z_list:
        W = np.array([apply_Mz(z, q) for q in Q])          # [k, n]
        out.append(Q.conj() @ W.T)
    return np.array(out)
