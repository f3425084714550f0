"""Host logic: the order in which the library's kernels carry out one
preconditioned CG step for small batches (the projected CG of Sec. III.A on
S P (H - e) P S), written out in numpy and checked against plain CG on the
same operator.

Per step the library's kernels do, in this order:
  first transform   beta = theta / rr (theta >= 0: a norm parked by the last
                    step), p = r + beta p, C = sum(slice sums of r) + beta C_old,
                    X = S p - Phi C   (= P S p)
  operator          Y = (H - e) X
  last transform    d = Re X^H Y  (= p^H S P Y, the outer projection after it),
                    rr = theta, theta = -1, C_old = C
  outer projection  Ap = S P Y
  x/r step          alpha = rr / d, x += alpha p, r -= alpha Ap,
                    slice sums of Phi^H S r, theta = |r|^2, flag
The initialisation leaves r = p = b, rr = |b|^2, theta = -1 and the slice sums
of b.  No GPU is involved: this pins the reordering itself (the recurrence of
the projector coefficients, the parked norm, p^H A p taken ahead of the outer
projection)."""
import numpy as np
import pytest


def _problem(n=160, nv=6, seed=0):
    rng = np.random.default_rng(seed)
    Phi, _ = np.linalg.qr(rng.standard_normal((n, nv)) + 1j * rng.standard_normal((n, nv)))
    P = np.eye(n) - Phi @ Phi.conj().T
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    H = X @ X.conj().T / n + np.diag(np.linspace(0.5, 6.0, n))
    S = 1.0 / np.sqrt(np.linspace(1.0, 4.0, n))
    b = S * (P @ (rng.standard_normal(n) + 1j * rng.standard_normal(n)))
    return Phi, P, H, S, b


def _plain_cg(A, b, tol, maxit=500):
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = np.vdot(r, r).real
    bb = rr
    for k in range(maxit):
        Ap = A(p)
        a = rr / np.vdot(p, Ap).real
        x = x + a * p
        r = r - a * Ap
        rn = np.vdot(r, r).real
        if rn <= tol * tol * bb:
            return x, k + 1
        p = r + (rn / rr) * p
        rr = rn
    raise AssertionError("plain CG did not converge")


def _library_order(Phi, P, H, S, b, tol, nsplit=5, maxit=500):
    n = len(b)
    chunk = -(-n // nsplit)
    slices = [slice(k * chunk, min(n, (k + 1) * chunk)) for k in range(nsplit)]

    def slice_sums(v):          # [nsplit][nv] partial sums of Phi^H (S v)
        return np.array([Phi[sl].conj().T @ (S[sl] * v[sl]) for sl in slices])

    x = np.zeros_like(b)
    r = b.copy()
    p = b.copy()
    part = slice_sums(b)
    rr = sum(np.vdot(b[sl], b[sl]).real for sl in slices)
    bb, theta, C_old = rr, -1.0, None
    drift = 0.0
    for k in range(maxit):
        # first transform
        upd = theta >= 0
        beta = theta / rr if upd else 0.0
        C = part.sum(0) + (beta * C_old if upd else 0.0)
        if upd:
            p = r + beta * p
        Xp = S * p - Phi @ C
        drift = max(drift, np.abs(Xp - P @ (S * p)).max() / np.abs(Xp).max())
        # operator and last transform
        Y = H @ Xp
        d = np.vdot(Xp, Y).real
        if theta >= 0:
            rr, theta = theta, -1.0
        C_old = C
        # outer projection and the x/r step
        Ap = S * (P @ Y)
        a = rr / d
        x = x + a * p
        r = r - a * Ap
        part = slice_sums(r)
        theta = sum(np.vdot(r[sl], r[sl]).real for sl in slices)
        if theta <= tol * tol * bb:
            return x, k + 1, drift
    raise AssertionError("library-order CG did not converge")


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_library_order_is_plain_cg(seed):
    Phi, P, H, S, b = _problem(seed=seed)
    A = lambda v: S * (P @ (H @ (P @ (S * v))))
    for tol in (1e-6, 1e-10):
        x1, k1 = _plain_cg(A, b, tol)
        x2, k2, drift = _library_order(Phi, P, H, S, b, tol)
        assert k1 == k2
        assert np.abs(x1 - x2).max() < 1e-11 * np.abs(x1).max()
        # the projector coefficients by recurrence stay those of P S p
        assert drift < 1e-11


def test_pAp_ahead_of_the_outer_projection():
    """p^H (S P Y) = (P S p)^H Y for any Y: the last transform may take the
    dot product before the outer projection."""
    Phi, P, H, S, _ = _problem(seed=4)
    rng = np.random.default_rng(9)
    p = rng.standard_normal(len(S)) + 1j * rng.standard_normal(len(S))
    Y = rng.standard_normal(len(S)) + 1j * rng.standard_normal(len(S))
    lhs = np.vdot(p, S * (P @ Y))
    rhs = np.vdot(P @ (S * p), Y)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
