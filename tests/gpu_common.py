"""Helpers shared by the GPU parity tests (inputs come from `synthetic`,
expected values from `oracle`; nothing here computes the method)."""
import numpy as np


def lib_order(lg, basis):
    """Index of each library sphere point in the oracle's sphere order."""
    pos = {tuple(m): i for i, m in enumerate(basis.m)}
    return np.array([pos[tuple(m)] for m in lg.sphere()])


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def colwise_rel(a, b):
    """max over leading index of |a_i - b_i| / |b_i|."""
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    return float(max(np.linalg.norm(a[i] - b[i]) / np.linalg.norm(b[i]) for i in range(a.shape[0])))


def tridiag_of(a, b):
    """The tridiagonal of a Lanczos run from its own coefficients (a library
    result checked against its own invariants, e.g. E(0) = T)."""
    a = np.asarray(a, dtype=float)
    k = len(a)
    b = np.asarray(b, dtype=float)[:k - 1]
    return np.diag(a) + np.diag(b, 1) + np.diag(b, -1)


def block_tridiag_of(A, B):
    """Block tridiagonal with diagonal blocks A_j and B_j below, B_j^H above
    (a library block-Lanczos result against its own invariants)."""
    A, B = np.asarray(A), np.asarray(B)
    nb, bs, _ = A.shape
    T = np.zeros((nb * bs, nb * bs), dtype=complex)
    for j in range(nb):
        T[j * bs:(j + 1) * bs, j * bs:(j + 1) * bs] = A[j]
        if j + 1 < nb:
            T[(j + 1) * bs:(j + 2) * bs, j * bs:(j + 1) * bs] = B[j]
            T[j * bs:(j + 1) * bs, (j + 1) * bs:(j + 2) * bs] = B[j].conj().T
    return T
