"""Closed-form chi0 of the free-electron box, V_loc = 0 (pin for the oracle).

With no potential the eigenstates are single plane waves e^{i K_m r}/sqrt(Omega)
with energies |K_m|^2/2, so each pair function of the Adler-Wiser sum (Sec. II)
is itself a plane wave and chi0 is diagonal in plane waves.  For a closed-shell
valence set V (no degenerate shell split) and x = e^{i K_q r} on the grid:

    chi0(z) x = lambda(q, z) x,
    lambda = (2/Omega) sum_{m_v in V} sum_{m_c in S \\ V, m_c = m_v - q mod N}
             [1/(z - D) - 1/(z + D)],  D = |K_c|^2/2 - |K_v|^2/2.

This enumerates integer triples only: no FFT, no diagonalisation.
"""
from __future__ import annotations

import itertools
import numpy as np


def sphere_triples(L: float, N: int, ecut: float):
    h = N // 2
    pts = []
    for m in itertools.product(range(-h + 1, h), repeat=3):
        e = 0.5 * (2 * np.pi / L) ** 2 * (m[0] ** 2 + m[1] ** 2 + m[2] ** 2)
        if e <= ecut:
            pts.append((m, e))
    return pts


def closed_shell_valence(pts, n_v: int):
    """The n_v lowest plane waves; raises if n_v splits a degenerate shell."""
    srt = sorted(pts, key=lambda t: t[1])
    if n_v < len(srt) and abs(srt[n_v][1] - srt[n_v - 1][1]) < 1e-12:
        raise ValueError("n_v splits a degenerate shell")
    return srt[:n_v], srt[n_v:]


def eigenvalue(L: float, N: int, ecut: float, n_v: int, q, z: complex) -> complex:
    pts = sphere_triples(L, N, ecut)
    val, con = closed_shell_valence(pts, n_v)
    con_map = {tuple(np.mod(m, N)): e for m, e in con}
    lam = 0.0 + 0.0j
    for mv, ev in val:
        key = tuple(np.mod(np.array(mv) - np.array(q), N))
        if key in con_map:
            D = con_map[key] - ev
            lam += 1.0 / (z - D) - 1.0 / (z + D)
    return 2.0 * lam / L ** 3
