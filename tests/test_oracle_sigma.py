"""Pins of the self-energy oracle (oracle/sigma.py) against what the paper and
the mathematics fix: the Lorentzian model's F_ne against numerical
quadrature of its definition, the free-electron box in closed form (Lindhard
eigenvalues, no diagonalisation), the sum-over-states forms against the
trace forms (completeness), the model term Sigma_A against the frequency
integral of sigma_N0 it stands for, the residue Lanczos against the dense
inverse, and the continuity in delta that Theta(0) = 1/2 provides."""
import numpy as np
import pytest
import scipy.integrate

from oracle import lanczos as olz
from oracle import lindhard
from oracle.pw import Basis
from oracle.sigma import (SigmaSOS, SigmaTrace, basis_W, gl_frequencies, lorentz_F, lorentz_f,
                          project_E)
from oracle.sos import SOS
from synthetic import make_workload, random_potentials


@pytest.mark.parametrize("alpha", [0.5, 1.0, 3.0])
def test_lorentz_F_is_the_integral_of_its_definition(alpha):
    for wne in (-2.0, -0.3, -1e-3, 1e-3, 0.05, 1.7):
        ref = scipy.integrate.quad(lambda w: lorentz_f(w, alpha) * wne / (w * w + wne * wne) / np.pi,
                                   0.0, np.inf, epsabs=1e-14, epsrel=1e-12, limit=400)[0]
        assert abs(lorentz_F(wne, alpha) - ref) < 1e-10 * max(1.0, abs(ref))
    assert lorentz_F(0.0, alpha) == 0.0


def test_lorentz_F_large_alpha_is_the_step_of_f_equal_one():
    # f = 1 (no model) gives F_ne = (Theta(w) - Theta(-w)) / 2 (Sec. III.B)
    for wne in (-0.7, 0.2, 3.0):
        assert abs(lorentz_F(wne, 1e9) - 0.5 * np.sign(wne)) < 1e-8


def test_gl_frequencies_integrate_the_half_line():
    w, wt = gl_frequencies(60)
    assert np.all(w > 0)
    assert abs(np.sum(wt / (1 + w * w)) - np.pi / 2) < 1e-12
    assert abs(np.sum(wt * np.exp(-w)) - 1.0) < 1e-10


@pytest.fixture(scope="module")
def c1():
    w = make_workload(1)
    b = Basis(w.L, w.N, w.ecut)
    s = SOS(b, w.V, w.n_v)
    _, _, Q, _ = olz.lanczos(lambda v: s.M(0.0, v), random_potentials(w.N, 1, 300)[0], 6)
    return w, b, s, Q


@pytest.mark.parametrize("e,delta", [(3, -0.07), (3, 0.2), (1, 0.03)])
def test_sum_over_states_equals_trace_forms(c1, e, delta):
    """Completeness (Sec. III.B): the sums over every eigenstate of Eqs. (dge),
    (dg0e), (dhe) equal the traces of Eq. (traces) with H inverted by linear
    solves, for a Lanczos basis that is far from complete."""
    w, b, s, Q = c1
    so = SigmaSOS(s, e, delta, alpha=1.0)
    tr = SigmaTrace(b, w.V, w.psi, w.eps, e, delta, alpha=1.0)
    assert abs(so.s - tr.s) < 1e-10
    W0 = basis_W(project_E(s.M, Q, 0.0))
    for x in (0.05, 0.7, 3.0):
        Wx = basis_W(project_E(s.M, Q, 1j * x))
        a, t = so.sigma_N(Q, Wx, x), tr.sigma_N(Q, Wx, x)
        assert abs(a - t) < 1e-11 * max(abs(a), 1e-3), (x, a, t)
        a, t = so.sigma_N0(Q, W0, x), tr.sigma_N0(Q, W0, x)
        assert abs(a - t) < 1e-11 * max(abs(a), 1e-3), (x, a, t)
    a, t = so.sigma_A(Q, W0), tr.sigma_A(Q, W0)
    assert abs(a - t) < 1e-11 * max(abs(a), 1e-3), (a, t)


def test_sigma_A_is_the_frequency_integral_of_sigma_N0(c1):
    """Eq. (dhe): Sigma_A = (1/pi) int_0^inf sigma_N0(i w) dw (the Lorentzian
    term is subtracted from the integrand and added back analytically)."""
    w, b, s, Q = c1
    so = SigmaSOS(s, 3, -0.07, alpha=1.0)
    W0 = basis_W(project_E(s.M, Q, 0.0))
    m = so._elements(Q, W0)
    nodes, wts = gl_frequencies(400)
    integral = sum(wt * lorentz_f(x, 1.0) * np.real(np.sum(m * so.wne / (x * x + so.wne ** 2)))
                   for x, wt in zip(nodes, wts)) / np.pi
    assert abs(integral - so.sigma_A(Q, W0)) < 1e-9 * abs(integral)


def test_free_box_closed_form():
    """V_loc = 0, one valence plane wave, e = that state: the pair functions
    are plane waves and eps - 1 is diagonal in plane waves with the Lindhard
    eigenvalues, so in a plane-wave basis Q
        sigma_N(i w) = sum_n v(K_n)/Omega W_{-n}(i w) wne/(w^2 + wne^2),
    W_m = 1/(1 + lambda_m) - 1, lambda_m = -v(K_m) chi0(K_m, i w)."""
    L, N, ecut = 10.0, 16, 6.0
    b = Basis(L, N, ecut)
    s = SOS(b, np.zeros((N, N, N)), 1)
    r = L * np.stack(np.meshgrid(*[np.arange(N)] * 3, indexing="ij"), -1).reshape(-1, 3) / N
    ms = [(1, 0, 0), (-1, 0, 0), (0, 1, 1), (0, -2, 1), (2, 1, 0), (0, 0, 0)]
    Q = np.array([np.exp(1j * (2 * np.pi / L) * r @ np.array(m, float)) for m in ms]) / np.sqrt(N ** 3)
    delta, alpha = -0.2, 1.0
    so = SigmaSOS(s, 0, delta, alpha)
    assert abs(so.s - delta) < 1e-12         # the free ground state has energy 0

    def v_of(m):
        k = 2 * np.pi / L * np.linalg.norm(m)
        return 2 * np.pi * (L / 2) ** 2 if k == 0 else 4 * np.pi * (1 - np.cos(k * L / 2)) / k ** 2

    def closed(x, kind):
        tot = 0.0
        for m in ms:
            n = tuple(-np.array(m))                 # the state n with -K_n = K_m
            en = 0.5 * (2 * np.pi / L) ** 2 * np.dot(n, n)
            if en > ecut:
                continue
            wne = en - so.s
            z = 1j * x if kind == "N" else 0.0
            lam = -v_of(m) * lindhard.eigenvalue(L, N, ecut, 1, m, z).real
            Wm = 1.0 / (1.0 + lam) - 1.0
            if kind == "A":
                fac = lorentz_F(wne, alpha)
            else:
                fac = wne / (x * x + wne * wne) * (lorentz_f(x, alpha) if kind == "N0" else 1.0)
            tot += v_of(n) / L ** 3 * Wm * fac
        return tot
    W0 = basis_W(project_E(s.M, Q, 0.0))
    for x in (0.1, 0.9):
        Wx = basis_W(project_E(s.M, Q, 1j * x))
        assert abs(so.sigma_N(Q, Wx, x) - closed(x, "N")) < 1e-12 * abs(closed(x, "N"))
        assert abs(so.sigma_N0(Q, W0, x) - closed(x, "N0")) < 1e-12 * abs(closed(x, "N0"))
    assert abs(so.sigma_A(Q, W0) - closed(0.0, "A")) < 1e-12 * abs(closed(0.0, "A"))


def test_residue_lanczos_converges_to_the_dense_inverse(c1):
    """Sec. VI: the residue element from a Lanczos recursion seeded with
    v^1/2 |v*e> converges to the exact <ev*| v^1/2 (eps^-1 - 1) v^1/2 |v*e>."""
    w, b, s, Q = c1
    so = SigmaSOS(s, 3, -0.05)
    poles = so.poles()
    assert [p[0] for p in poles] == [3] and poles[0][1:] == (1.0, -1.0)
    om = float(so.wne[3])
    exact = so.residue_element(3, om, None)
    assert exact < 0.0                           # eps^-1 - 1 <= 0 below the first excitation
    errs = [abs(so.residue_element(3, om, k) - exact) / abs(exact) for k in (2, 4, 40)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-10, errs


def test_theta_half_keeps_sigma_continuous_in_delta():
    """Footnote of Sec. III.B: with Theta(0) = 1/2 the jumps of Sigma_A and
    Sigma_P as delta crosses eps_m - eps_e cancel (complete basis, exact
    inverse), while each term jumps by the full matrix element.  A small box
    (8^3 grid) keeps the dense inverses cheap."""
    w = make_workload(1, N=8, L=6.0, ecut=3.0)
    b = Basis(w.L, w.N, w.ecut)
    s = SOS(b, w.V, w.n_v)
    Q = np.eye(b.N ** 3, dtype=np.complex128)   # complete basis: W(0) = eps^-1(0) - 1
    e, m = 3, 2                                 # cross the pole of valence state m
    dm = s.eps[m] - s.eps[e]
    W0 = basis_W(s.M_matrix(0.0))
    vals = []
    for h in (-1e-7, 0.0, 1e-7):
        so = SigmaSOS(s, e, dm + h)
        vals.append((so.sigma_A(Q, W0), so.sigma_P(None)))
    jumpA = vals[2][0] - vals[0][0]
    jumpP = vals[2][1] - vals[0][1]
    assert abs(jumpA) > 1e-3 and abs(jumpP) > 1e-3
    assert abs(jumpA + jumpP) < 1e-5 * abs(jumpA)
    tot = [a + p for a, p in vals]
    assert abs(tot[1] - 0.5 * (tot[0] + tot[2])) < 1e-5 * abs(jumpA)
