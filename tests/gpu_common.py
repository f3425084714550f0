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
