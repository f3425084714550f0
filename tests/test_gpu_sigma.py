"""GPU parity of the self-energy calls (lgw_sigma_traces, lgw_sigma_residues)
against the oracle's sum-over-states forms, on the c1-size system.

Each side builds its own static Lanczos basis from the same seed (Sec. IV);
the bases are compared first, then the traces sigma_N(i w), sigma_N0(i w)
and the Lorentzian term Sigma_A (Secs. III.B, IV), and the residue term
Sigma_P from four real-frequency Lanczos steps per pole (Sec. VI), all in
FP64 at 1e-10 relative to the largest value of each set."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import lanczos as olz
from oracle.pw import Basis
from oracle.sigma import SigmaSOS, basis_W, project_E
from oracle.sos import SOS
from synthetic import make_workload, random_potentials
from tests.gpu_common import colwise_rel

WS = [0.05, 0.4, 1.3, 4.0]
CASES = [(3, -0.07), (3, 0.2), (1, 0.03)]


@pytest.fixture(scope="module")
def c1sig():
    from paper_1408_3036_amd import Lgw
    w = make_workload(1)
    b = Basis(w.L, w.N, w.ecut)
    s = SOS(b, w.V, w.n_v)
    lg = Lgw(w.L, w.N, w.ecut, torch.from_numpy(w.V), torch.from_numpy(w.psi), w.eps, tol=1e-13)
    q0 = random_potentials(w.N, 1, 310)[0]
    k = w.lanczos_steps
    _, _, Q, kd = lg.lanczos(torch.from_numpy(q0), k)
    _, _, RQ, rkd = olz.lanczos(lambda v: s.M(0.0, v), q0, k)
    assert kd == rkd == k
    yield w, b, s, lg, Q, RQ
    lg.close()


def test_sigma_bases_agree(c1sig):
    w, b, s, lg, Q, RQ = c1sig
    assert colwise_rel(Q.cpu().numpy(), RQ) < 1e-10


@pytest.mark.parametrize("e,delta", CASES)
def test_sigma_traces_match_oracle(c1sig, e, delta):
    w, b, s, lg, Q, RQ = c1sig
    sN, sN0, sA = lg.sigma_traces(e, delta, Q, WS, alpha=1.0)
    so = SigmaSOS(s, e, delta, alpha=1.0)
    W0 = basis_W(project_E(s.M, RQ, 0.0))
    rN = np.array([so.sigma_N(RQ, basis_W(project_E(s.M, RQ, 1j * x)), x) for x in WS])
    rN0 = np.array([so.sigma_N0(RQ, W0, x) for x in WS])
    rA = so.sigma_A(RQ, W0)
    eN = np.abs(sN - rN).max() / np.abs(rN).max()
    eN0 = np.abs(sN0 - rN0).max() / np.abs(rN0).max()
    eA = abs(sA - rA) / abs(rA)
    print(f"sigma e={e} delta={delta}: sigma_N {sN} (rel {eN:.1e}), sigma_N0 rel {eN0:.1e}, "
          f"Sigma_A {sA:.10f} (rel {eA:.1e})")
    assert eN < 1e-10 and eN0 < 1e-10 and eA < 1e-10


@pytest.mark.parametrize("e,delta", CASES + [(3, 0.0)])
def test_sigma_residues_match_oracle(c1sig, e, delta):
    w, b, s, lg, Q, RQ = c1sig
    sp, npl = lg.sigma_residues(e, delta, k_p=4)
    so = SigmaSOS(s, e, delta)
    poles = so.poles()
    assert npl == len(poles)
    ref = so.sigma_P(4)
    exact = so.sigma_P(None) if npl else 0.0
    print(f"Sigma_P e={e} delta={delta}: {npl} poles, library {sp:.12f}, oracle (4 steps) {ref:.12f}, "
          f"dense inverse {exact:.12f}")
    if npl == 0:
        assert sp == 0.0
    else:
        assert abs(sp - ref) < 1e-10 * abs(ref)
