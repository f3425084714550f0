"""Writes tests/golden/c5_oracle.json for the differentiation workload
(silane-48: 64 Lanczos vectors of eps(0) - 1 from the seeded q0, the loss
L = sum_z log det(I + E(z)) over z = 0 and four imaginary frequencies,
Sec. IV basis reused at every frequency as in Sec. VI):

  * the oracle's loss at the workload's potential;
  * its Richardson-extrapolated central differences along two seeded smooth
    directions d (step h and 2h), the ground state recomputed at every
    displaced potential, i.e. the total derivative dL/dV_loc . d.

Calls only oracle/ and the seeded inputs of synthetic/ (no library code);
it runs once on the CPU, one worker process per loss evaluation:

    python tests/golden/make_c5_oracle.py [workers]
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

K = 64
Q0_SEED = 73
DIR_SEED = 74
H = 1e-2


def freqs():
    return [0.0] + list(1j * np.geomspace(0.1, 2.0, 4))


def _loss(task):
    label, scale, direction = task
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except ImportError:
        pass
    sys.path.insert(0, ROOT)
    from oracle.lanczos import logdet_loss
    from oracle.pw import Basis
    from oracle.sternheimer import MatrixFree
    from synthetic import ground_state, make_workload, random_potentials, smooth_directions
    w = make_workload(2)
    V = w.V.copy()
    if direction is not None:
        V = V + scale * smooth_directions(w.N, w.L, DIR_SEED, 2)[direction]
    t = time.time()
    psi, eps, _ = ground_state(V, w.L, w.ecut, w.n_v)
    mf = MatrixFree(Basis(w.L, w.N, w.ecut), V, psi, eps, rtol=1e-13)
    q0 = random_potentials(w.N, 1, Q0_SEED)[0]
    L = logdet_loss(mf.M, q0, K, freqs())
    print(f"{label}: L = {L:.15f} ({time.time() - t:.0f}s)", flush=True)
    return label, L


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else min(9, os.cpu_count() or 1)
    tasks = [("base", 0.0, None)]
    for i in range(2):
        for s in (1, -1, 2, -2):
            tasks.append((f"d{i}{'+' if s > 0 else '-'}{abs(s)}h", s * H, i))
    with mp.get_context("spawn").Pool(workers) as pool:
        res = dict(pool.map(_loss, tasks, chunksize=1))
    dirs = []
    for i in range(2):
        f1 = (res[f"d{i}+1h"] - res[f"d{i}-1h"]) / (2 * H)
        f2 = (res[f"d{i}+2h"] - res[f"d{i}-2h"]) / (4 * H)
        dirs.append({"index": i, "losses": {k: res[k] for k in res if k.startswith(f"d{i}")},
                     "central_h": f1, "central_2h": f2, "richardson": (4 * f1 - f2) / 3})
    out = {"workload": "silane-48 (L = 20 bohr, 48^3, ecut 10 Ha, N_v = 4)", "k": K,
           "z_imag": [float(np.imag(z)) for z in freqs()], "q0_seed": Q0_SEED,
           "directions": "synthetic.smooth_directions(N, L, 74, 2)", "h": H,
           "loss": res["base"], "dL_dV_dot_d": dirs,
           "how": "oracle.lanczos.logdet_loss with the matrix-free FP64 Sternheimer chi0 (CG, rtol 1e-13); "
                  "ground state recomputed at each displaced potential by synthetic.ground_state"}
    with open(os.path.join(HERE, "c5_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
