"""Writes tests/golden/lanczos520_oracle.json: the Lanczos coefficients of
eps(0) - 1 = -v^(1/2) chi0(0) v^(1/2) on the small box (16^3 grid, 739 plane
waves, 4 valence bands) over 520 steps from the seeded q0, with full
reorthogonalization (two classical Gram-Schmidt passes per step, Sec. IV).

520 steps take the library's recursion past its fused Gram-Schmidt form,
which holds at most 512 earlier vectors; the oracle needs about a minute for
them, too long for a test, so the coefficients are stored.  A 1e-14 relative
perturbation of q0 moves no coefficient by more than 1.3e-14 of max |alpha|
(the recursion is well conditioned here).

Calls only oracle/ and the seeded inputs of synthetic/ (no library code):

    python tests/golden/make_lanczos520_oracle.py
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

K = 520
Q0_SEED = 97


def main() -> None:
    from oracle import lanczos as olz
    from oracle.pw import Basis
    from oracle.sos import SOS
    from synthetic import make_workload, random_potentials
    w = make_workload(1)
    s = SOS(Basis(w.L, w.N, w.ecut), w.V, w.n_v)
    q0 = random_potentials(w.N, 1, Q0_SEED)[0]
    t = time.time()
    alpha, beta, _, k_done = olz.lanczos(lambda v: s.M(0.0, v), q0, K)
    out = {
        "workload": "small box (make_workload(1)): 16^3 grid, 739 plane waves, 4 valence bands",
        "operator": "eps(0) - 1 = -v^1/2 chi0(0) v^1/2, sum-over-states oracle (oracle/sos.py)",
        "q0": f"random_potentials(16, 1, {Q0_SEED})[0]",
        "k": K,
        "k_done": int(k_done),
        "alpha": [float(a) for a in alpha[:k_done]],
        "beta": [float(b) for b in beta[:k_done]],
        "seconds": round(time.time() - t, 1),
    }
    with open(os.path.join(HERE, "lanczos520_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=0)
    print(f"k_done {k_done}, {out['seconds']} s")


if __name__ == "__main__":
    main()
