"""Workspace poisoning: with LGW_POISON=1 every workspace buffer of the
library starts filled with NaN bytes, so a kernel that reads workspace it
never wrote (a stale tail of a ragged tile, an unset padding lane, a
partial sum slot no launch filled) turns its outputs into NaN.  The main
paths run in a child process with the variable set (it is read once per
process) and must still match the oracle."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
sys.path.insert(0, ROOT)
import numpy as np, torch
from paper_1408_3036_amd import Lgw
from oracle.pw import Basis
from oracle.sos import SOS
from oracle import lanczos as olz
from oracle.sigma import SigmaSOS, basis_W, project_E
from synthetic import make_workload, random_potentials

def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))

w = make_workload(1)
s = SOS(Basis(w.L, w.N, w.ecut), w.V, w.n_v)
out = {}
x = random_potentials(w.N, 3, 41)
zs = [0.0, 0.3j, 0.5 + 0.0036749j]
ref = [s.chi0(z, x) for z in zs]
for name, kw in [("fp64", {}), ("mixed", dict(precision="mixed", tol=1e-10)),
                 ("fast", dict(precond=True, imag_form="shifted")),
                 ("multishift", dict(multishift=True)),
                 ("mixed_fast_ms", dict(precision="mixed", tol=1e-10, precond=True, imag_form="shifted",
                                        multishift=True))]:
    lg = Lgw(w.L, w.N, w.ecut, torch.from_numpy(w.V), torch.from_numpy(w.psi), w.eps, **kw)
    dn = lg.chi0_apply(torch.from_numpy(x), zs).cpu().numpy()
    out["chi0_" + name] = max(rel(dn[k], ref[k]) for k in range(len(zs)))
    q0 = random_potentials(w.N, 1, 42)[0]
    a, b, Q, E, kd = lg.lanczos_project(torch.from_numpy(q0), 6, [0.0, 0.4j])
    ra, rb, RQ, _ = olz.lanczos(lambda v: s.M(0.0, v), q0, 6)
    Eref = olz.project(lambda z, v: s.M(z, v), RQ, [0.0, 0.4j])
    out["lanczos_alpha_" + name] = float(np.abs(a.cpu().numpy() - ra).max() / np.abs(ra).max())
    out["project_" + name] = max(rel(E.cpu().numpy()[k], Eref[k]) for k in range(2))
    lg.close()
lg = Lgw(w.L, w.N, w.ecut, torch.from_numpy(w.V), torch.from_numpy(w.psi), w.eps)
Q0 = random_potentials(w.N, 2, 43)
A, B, BQ, nd = lg.block_lanczos(torch.from_numpy(Q0), 2)
RA, RB, RBQ = olz.block_lanczos(lambda v: s.M(0.0, v), Q0, 2)[:3]
out["block_A"] = rel(A.cpu().numpy()[:nd], np.asarray(RA)[:nd])
_, _, RQ, _ = olz.lanczos(lambda v: s.M(0.0, v), random_potentials(w.N, 1, 44)[0], 6)
ws = np.array([0.2, 1.1])
sN, sN0, sA = lg.sigma_traces(3, -0.07, torch.from_numpy(RQ), ws, alpha=1.0)
so = SigmaSOS(s, 3, -0.07, alpha=1.0)
Wz = [basis_W(project_E(s.M, RQ, 1j * v)) for v in ws]
out["sigma_N"] = max(abs(sN[i] - so.sigma_N(RQ, Wz[i], ws[i])) / abs(so.sigma_N(RQ, Wz[i], ws[i])) for i in range(2))
lg.close()
print("RESULT " + json.dumps(out))
""".replace("ROOT", repr(ROOT))


def test_paths_read_no_unwritten_workspace(tmp_path):
    script = tmp_path / "child.py"
    script.write_text(CHILD)
    env = dict(os.environ, LGW_POISON="1")
    r = subprocess.run([sys.executable, str(script)], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    line = [l for l in r.stdout.splitlines() if l.startswith("RESULT ")][-1]
    res = json.loads(line[len("RESULT "):])
    print(res)
    for k, v in res.items():
        bar = 1e-6 if "mixed" in k else 1e-10
        assert v == v and v < bar, (k, v)       # v == v: not NaN
