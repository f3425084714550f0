"""Build and store the boxes of the batched uneven-systems workload over the
host cores (input generation only: ground states of synthetic potentials).

Boxes are stored as .npy files so that several processes can read them
without pickling large orbitals."""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np


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
    from synthetic.workloads import make_workload
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
