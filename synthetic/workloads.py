"""Workload recipes: box, grid, cut-off, Gaussian-well potential, seeds.

Every random draw comes from ``numpy.random.default_rng([14083036, cfg, sys,
attempt])`` so that a workload is a pure function of its indices.
"""
from __future__ import annotations

import dataclasses
import numpy as np

SEED_BASE = 14083036
HA_PER_EV = 1.0 / 27.211386245988   # 1 eV in hartree


@dataclasses.dataclass
class Workload:
    """One synthetic molecule-in-a-box system and the work to run on it."""
    name: str
    L: float                 # cubic box edge, bohr
    N: int                   # grid points per axis
    ecut: float              # plane-wave cut-off, Ha (0.5*|G|^2 <= ecut)
    n_v: int                 # valence bands
    n_wells: int
    V: np.ndarray            # [N,N,N] float64 local potential, Ha
    psi: np.ndarray | None   # [n_v, N^3] complex128 grid orbitals
    eps: np.ndarray | None   # [n_v] float64, ascending
    gap: float | None        # eps[n_v] - eps[n_v-1]
    lanczos_steps: int
    z: np.ndarray            # complex frequencies (0,w)=i*w, (w,eta) real axis
    seed: tuple


def imag_freqs(n: int, wmin: float = 0.01, wmax: float = 2.0) -> np.ndarray:
    """{0} followed by n-1 log-spaced imaginary frequencies i*w, w in [wmin, wmax] Ha."""
    w = np.concatenate([[0.0], np.geomspace(wmin, wmax, n - 1)]) if n > 1 else np.zeros(1)
    return 1j * w


def real_freqs(n: int, wmax: float = 1.0, eta_ev: float = 0.1) -> np.ndarray:
    """n real frequencies linspace(0, wmax) Ha with broadening eta (in eV) as w + i*eta."""
    return np.linspace(0.0, wmax, n) + 1j * eta_ev * HA_PER_EV


def gaussian_wells(L: float, N: int, n_wells: int, rng: np.random.Generator,
                   depth=(1.0, 4.0), width=(0.8, 1.5), radius=2.0) -> np.ndarray:
    """Sum of attractive periodic Gaussian wells sampled on the grid r_n = L*n/N.

    V(r) = -sum_i D_i sum_{T in {-1,0,1}^3} exp(-|r - R_i - L T|^2 / (2 s_i^2)),
    D_i ~ U(depth), s_i ~ U(width), R_i = box centre + radius * u^(1/3) * g/|g|
    with g ~ N(0, I3) and u ~ U(0,1) (uniform in the ball).  Draw order: D, s, g, u.
    """
    D = rng.uniform(depth[0], depth[1], n_wells)
    s = rng.uniform(width[0], width[1], n_wells)
    g = rng.standard_normal((n_wells, 3))
    u = rng.uniform(0.0, 1.0, n_wells)
    centres = L / 2 + radius * np.cbrt(u)[:, None] * g / np.linalg.norm(g, axis=1)[:, None]
    x = L * np.arange(N) / N
    V = np.zeros((N, N, N))
    for i in range(n_wells):
        # separable Gaussian: product of three 1D periodic sums
        fac = []
        for a in range(3):
            d = x[:, None] - centres[i, a] - L * np.array([-1.0, 0.0, 1.0])[None, :]
            fac.append(np.exp(-d ** 2 / (2 * s[i] ** 2)).sum(axis=1))
        V -= D[i] * np.einsum("i,j,k->ijk", fac[0], fac[1], fac[2])
    return V


def random_potentials(N: int, n: int, seed, real: bool = True) -> np.ndarray:
    """n random perturbing potentials on the grid, each Euclidean-normalised.

    real=True: N(0,1) per grid point (imaginary part zero); else complex Gaussian.
    Returned as complex128 [n, N^3].
    """
    rng = np.random.default_rng(seed)
    if real:
        x = rng.standard_normal((n, N ** 3)).astype(np.complex128)
    else:
        x = rng.standard_normal((n, N ** 3)) + 1j * rng.standard_normal((n, N ** 3))
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def smooth_directions(N: int, L: float, seed, n: int, n_bumps: int = 3, width: float = 1.5) -> list:
    """n smooth real potential displacements on the N^3 grid of an L box (for
    directional derivatives): each a sum of n_bumps periodic Gaussian bumps of
    the given width, centres uniform in the box, N(0,1) amplitudes; draws
    from default_rng(seed) in the order centre, amplitude per bump."""
    rng = np.random.default_rng(seed)
    r = L * np.stack(np.meshgrid(*[np.arange(N)] * 3, indexing="ij"), -1) / N
    out = []
    for _ in range(n):
        d = np.zeros((N,) * 3)
        for _ in range(n_bumps):
            c = rng.uniform(0, L, 3)
            dd = (r - c + L / 2) % L - L / 2
            d += rng.standard_normal() * np.exp(-np.sum(dd ** 2, -1) / (2 * width ** 2))
        out.append(d)
    return out


# (L, N, ecut, n_wells, n_v, lanczos_steps, frequency recipe)
CONFIGS = {
    1: dict(name="tiny-16", L=10.0, N=16, ecut=6.0, n_wells=5, n_v=4, lanczos=8,
            z="static"),
    2: dict(name="silane-48", L=20.0, N=48, ecut=10.0, n_wells=5, n_v=4, lanczos=64,
            z="c2"),
    3: dict(name="large-72", L=24.0, N=72, ecut=15.0, n_wells=20, n_v=16, lanczos=256,
            z="c3"),
}


def config_freqs(kind: str) -> np.ndarray:
    if kind == "static":
        return np.zeros(1, dtype=np.complex128)
    if kind == "c2":
        return np.concatenate([imag_freqs(16), real_freqs(16)])
    if kind == "c3":
        return imag_freqs(32)
    if kind == "uneven":
        return imag_freqs(8)
    raise ValueError(kind)


def make_workload(cfg: int, sys: int = 0, with_ground_state: bool = True,
                  max_attempts: int = 20, **override) -> Workload:
    """Build config `cfg` deterministically (1..3; 4 = box `sys` of the uneven
    batch, see uneven_box_params); reseed until the gap is >= 1e-3 Ha."""
    p = dict(CONFIGS[cfg]) if cfg != 4 else uneven_box_params(sys)
    p.update(override)
    # a box of the uneven batch whose drawn N_v would split a degenerate level
    # (few wells: the upper states are the box's free-particle shells) takes
    # the closed shell below it, the largest n <= N_v (n >= 2) with a gap
    shell_down = cfg == 4 and "n_v" not in override
    for attempt in range(max_attempts):
        seed = (SEED_BASE, cfg, sys, attempt)
        rng = np.random.default_rng(list(seed))
        V = gaussian_wells(p["L"], p["N"], p["n_wells"], rng)
        psi = eps = gap = None
        if with_ground_state:
            from .ground_state import ground_state
            psi, eps, eps_all = ground_state(V, p["L"], p["ecut"], p["n_v"])
            gap = float(eps_all[p["n_v"]] - eps_all[p["n_v"] - 1])
            if gap < 1e-3 and shell_down:
                n = p["n_v"] - 1
                while n >= 2 and eps_all[n] - eps_all[n - 1] < 1e-3:
                    n -= 1
                if n >= 2:
                    p["n_v"] = n
                    psi, eps = psi[:n].copy(), eps[:n].copy()
                    gap = float(eps_all[n] - eps_all[n - 1])
            if gap < 1e-3:
                continue
        return Workload(name=p["name"], L=p["L"], N=p["N"], ecut=p["ecut"], n_v=p["n_v"],
                        n_wells=p["n_wells"], V=V, psi=psi, eps=eps, gap=gap,
                        lanczos_steps=p["lanczos"], z=config_freqs(p["z"]), seed=seed)
    raise RuntimeError("no seed with a valence/conduction gap >= 1e-3 Ha")


def uneven_box_params(sys: int) -> dict:
    """Recipe of one box of the batched uneven-systems workload: grid N drawn
    from {24, 32, 40, 48, 64}, edge L = N * 20/48 bohr (the silane-48 ratio of
    grid to box), ecut 10 Ha, N_v from 2..32, 1..12 wells; 8 imaginary
    frequencies; 32 Lanczos steps.  Draws come from default_rng([14083036, 4,
    sys]) in the order N, N_v, wells (the potential itself is drawn by
    make_workload from its own seed)."""
    rng = np.random.default_rng([SEED_BASE, 4, sys])
    N = int(rng.choice([24, 32, 40, 48, 64]))
    n_v = int(rng.integers(2, 33))
    n_wells = int(rng.integers(1, 13))
    return dict(name=f"uneven-{sys}", L=N * 20.0 / 48.0, N=N, ecut=10.0, n_wells=n_wells,
                n_v=n_v, lanczos=32, z="uneven")
