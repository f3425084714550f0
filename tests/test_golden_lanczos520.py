"""The stored 520-step oracle recursion (tests/golden/lanczos520_oracle.json,
written by make_lanczos520_oracle.py from oracle/ alone) against the oracle
itself: its first steps equal a fresh short oracle run from the same seed."""
import json
import os

import numpy as np

from oracle import lanczos as olz
from oracle.pw import Basis
from oracle.sos import SOS
from synthetic import make_workload, random_potentials

HERE = os.path.dirname(os.path.abspath(__file__))


def test_stored_recursion_starts_as_the_oracle():
    d = json.load(open(os.path.join(HERE, "golden", "lanczos520_oracle.json")))
    assert d["k"] == d["k_done"] == len(d["alpha"]) == len(d["beta"]) == 520
    w = make_workload(1)
    s = SOS(Basis(w.L, w.N, w.ecut), w.V, w.n_v)
    q0 = random_potentials(w.N, 1, 97)[0]
    ra, rb, _, kd = olz.lanczos(lambda v: s.M(0.0, v), q0, 12)
    assert kd == 12
    a, b = np.array(d["alpha"][:12]), np.array(d["beta"][:12])
    assert np.abs(a - ra).max() <= 1e-13 * np.abs(ra).max()
    assert np.abs(b - rb).max() <= 1e-13 * np.abs(ra).max()
