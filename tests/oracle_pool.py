"""Run the oracle's matrix-free Sternheimer chi0 (O2) over the host cores.

Test infrastructure: a process pool whose workers each solve the Sternheimer
systems of single valence bands with the oracle and return that band's
contribution to chi0(z) x (the oracle sums bands; the caller adds the
returned contributions).  Box data are passed as .npy files, memory-mapped
by the workers, so that large boxes are not pickled once per task.  Nothing
here computes the method itself."""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from synthetic.boxes import host_workers, make_uneven_boxes, save_box  # noqa: F401  (re-exported)

_CACHE: dict = {}


def _box(pre: str):
    if pre not in _CACHE:
        import sys
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        if root not in sys.path:
            sys.path.insert(0, root)
        from oracle.pw import Basis
        from oracle.sternheimer import MatrixFree
        L, N, ecut = np.load(pre + "_meta.npy")
        b = Basis(float(L), int(N), float(ecut))
        mf = MatrixFree(b, np.load(pre + "_V.npy"), np.load(pre + "_psi.npy", mmap_mode="r"),
                        np.load(pre + "_eps.npy"))
        _CACHE.clear()
        _CACHE[pre] = mf
    return _CACHE[pre]


def _band_task(task):
    """Band v's part of chi0(z) x at each z: -2 psi_v Scatter(f_v(z))."""
    pre, v, zs, x = task
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except ImportError:
        pass
    mf = _box(pre)
    psi_v = np.asarray(mf.psi_v[v])
    b = mf.P(mf.b.gather(psi_v.conj() * x))
    return [-2.0 * psi_v * mf.b.scatter(mf.solve_band(v, complex(z), b)) for z in zs]


def chi0_by_bands(jobs, workers: int | None = None):
    """jobs: list of (prefix, n_v, zs, x).  Returns, per job, chi0(z) x for
    each z [n_z, N^3], the band solves spread over worker processes."""
    tasks, owner = [], []
    for j, (pre, nv, zs, x) in enumerate(jobs):
        for v in range(nv):
            tasks.append((pre, v, list(zs), np.asarray(x)))
            owner.append(j)
    order = sorted(range(len(tasks)), key=lambda i: tasks[i][0])   # a box's bands together
    ctx = mp.get_context("spawn")
    out = [None] * len(jobs)
    with ctx.Pool(processes=workers or host_workers()) as pool:
        res = pool.map(_band_task, [tasks[i] for i in order], chunksize=1)
    for i, r in zip(order, res):
        j = owner[i]
        r = np.array(r)
        out[j] = r if out[j] is None else out[j] + r
    return out

