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

_CACHE: dict = {}


def host_workers() -> int:
    """Worker processes: the cores this process may use, at most 16."""
    return max(1, min(len(os.sched_getaffinity(0)), 16))


def save_box(d: str, key: str, L: float, N: int, ecut: float, V, psi, eps) -> str:
    """Store one box's inputs under directory d; returns the path prefix."""
    pre = os.path.join(d, key)
    np.save(pre + "_V.npy", np.asarray(V, dtype=np.float64))
    np.save(pre + "_psi.npy", np.asarray(psi, dtype=np.complex128))
    np.save(pre + "_eps.npy", np.asarray(eps, dtype=np.float64))
    np.save(pre + "_meta.npy", np.array([L, N, ecut], dtype=np.float64))
    return pre


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


def _make_box(task):
    """Build box `sys` of the uneven batch and store it; returns its sizes."""
    d, sys_i, threads = task
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=threads)
    except ImportError:
        pass
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from synthetic import make_workload
    w = make_workload(4, sys=sys_i)
    pre = save_box(d, f"box{sys_i:02d}", w.L, w.N, w.ecut, w.V, w.psi, w.eps)
    return dict(sys=sys_i, pre=pre, L=w.L, N=w.N, ecut=w.ecut, n_v=w.n_v, n_wells=w.n_wells,
                gap=w.gap, z=np.asarray(w.z))


def make_uneven_boxes(d: str, n: int = 32, workers: int | None = None):
    """All n boxes of the uneven batch, built in worker processes and stored
    under d (synthetic inputs only); returns their descriptions.  A quarter of
    the cores run boxes side by side, each with four BLAS threads (the small
    boxes' dense eigensolver uses them), largest grids first."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from synthetic.workloads import uneven_box_params
    cores = workers or host_workers()
    procs = max(1, cores // 4)
    order = sorted(range(n), key=lambda i: -uneven_box_params(i)["N"])
    ctx = mp.get_context("spawn")
    with ctx.Pool(processes=procs) as pool:
        res = pool.map(_make_box, [(d, i, max(1, cores // procs)) for i in order], chunksize=1)
    return sorted(res, key=lambda r: r["sys"])
