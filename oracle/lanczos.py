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


def logdet_loss(apply_Mz, q0: np.ndarray, k: int, z_list) -> float:
    """Scalar summary of the frequency-dependent dielectric matrix in the static
    basis: L = sum_z log det(I + E(z)) = sum_z sum_i log(1 + theta_i(z)), with
    E(z) = Q^H (eps(z) - 1) Q over the k Lanczos vectors of eps(0) - 1 from q0
    (Sec. IV basis, reused at every imaginary frequency as in Sec. VI).  E(z)
    is Hermitian on the imaginary axis and eps - 1 is positive semidefinite
    there, so I + E(z) is positive definite."""
    _, _, Q, _ = lanczos(lambda x: apply_Mz(0.0, x), q0, k)
    total = 0.0
    for Ez in project(apply_Mz, Q, z_list):
        S = np.eye(len(Q)) + 0.5 * (Ez + Ez.conj().T)
        sign, ld = np.linalg.slogdet(S)
        if not np.real(sign) > 0:
            raise ValueError("I + E(z) is not positive definite")
        total += float(ld)
    return total


def eps_inverse_in_basis(E: np.ndarray) -> np.ndarray:
    """(I + E(z))^-1 for every E(z) = Q^H (eps(z) - 1) Q of a list [n_z, k, k]
    (Sec. IV: the dielectric matrix inverted in the small basis; eps^-1 within
    span(Q) is 1 + Q ((I + E)^-1 - I) Q^H)."""
    E = np.asarray(E)
    k = E.shape[-1]
    return np.array([np.linalg.inv(np.eye(k) + e) for e in E.reshape(-1, k, k)])


def ritz_values(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """Ritz values of the Lanczos recursion (Sec. IV): the eigenvalues of the
    tridiagonal T, ascending."""
    return np.linalg.eigvalsh(tridiag(alpha, beta))


def _qr_pos(W: np.ndarray):
    """Thin QR of the columns of W (n x b) with a non-negative diagonal of R."""
    Qf, R = np.linalg.qr(W)
    d = np.sign(np.real(np.diag(R)))
    d[d == 0] = 1.0
    return Qf * d[None, :], R * d[:, None]


def block_lanczos(apply_M, Q0: np.ndarray, nblk: int, deflate: float = 1e-10):
    """Block Lanczos with full reorthogonalisation on Hermitian M.

    Sec. IV builds a Krylov basis with one starting vector; its block form
    starts from b vectors (rows of Q0), so that each step applies M to b
    vectors at once:

        Q_0 R_0 = Q0^T (thin QR),  B_{-1} = 0
        W = M Q_j;  A_j = Q_j^H W (Hermitian part);  W -= Q_j A_j + Q_{j-1} B_{j-1}^H
        W -= Q (Q^H W)  (twice, against every previous block)
        Q_{j+1} B_j = W  (thin QR, non-negative diagonal)

    so that M Q_j = Q_{j-1} B_{j-1}^H + Q_j A_j + Q_{j+1} B_j.  A column whose
    norm after reorthogonalisation falls below `deflate` times the block norm
    is deflated: its row of B_j is zero and a fresh direction (a fixed-seed
    random vector orthogonalised against the basis) replaces it.
    Returns (A [nblk, b, b], B [nblk, b, b], Q [nblk*b, n]).
    """
    Q0 = np.asarray(Q0, dtype=np.complex128)
    b, n = Q0.shape
    Qj, _ = _qr_pos(Q0.T)                       # n x b
    blocks = [Qj]
    As, Bs = [], []
    Bprev = None
    rng = np.random.default_rng(12345)
    for j in range(nblk):
        W = np.stack([apply_M(Qj[:, k]) for k in range(b)], axis=1)
        Aj = Qj.conj().T @ W
        Aj = 0.5 * (Aj + Aj.conj().T)
        W = W - Qj @ Aj
        if Bprev is not None:
            W = W - blocks[-2] @ Bprev.conj().T
        Qall = np.concatenate(blocks, axis=1)
        for _ in range(2):
            W = W - Qall @ (Qall.conj().T @ W)
        wn = np.linalg.norm(W)
        Qn, Bj = _qr_pos(W)
        for k in range(b):
            if abs(Bj[k, k]) < deflate * max(wn, 1e-300):
                Bj[k, :] = 0.0
                r = rng.standard_normal(n) + 0j
                Qc = np.concatenate([Qall, Qn[:, :k]], axis=1)
                for _ in range(2):
                    r = r - Qc @ (Qc.conj().T @ r)
                Qn[:, k] = r / np.linalg.norm(r)
        As.append(Aj)
        Bs.append(Bj)
        if j + 1 < nblk:
            blocks.append(Qn)
            Qj = Qn
        Bprev = Bj
    return np.array(As), np.array(Bs), np.concatenate(blocks, axis=1).T


def block_tridiag(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Dense block-tridiagonal T: diagonal blocks A_j, T[j+1, j] = B_j, T[j, j+1] = B_j^H."""
    nb, b, _ = A.shape
    T = np.zeros((nb * b, nb * b), dtype=np.complex128)
    for j in range(nb):
        T[j * b:(j + 1) * b, j * b:(j + 1) * b] = A[j]
        if j + 1 < nb:
            T[(j + 1) * b:(j + 2) * b, j * b:(j + 1) * b] = B[j]
            T[j * b:(j + 1) * b, (j + 1) * b:(j + 2) * b] = B[j].conj().T
    return T
