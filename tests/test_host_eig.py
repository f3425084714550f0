"""Host logic: the library's small Hermitian eigensolver (csrc/herm_eig.h),
compiled with g++ into a tiny driver and compared with numpy.linalg.eigh on
random, degenerate, diagonal and tiny matrices.  The driver is built twice:
plain, and with AddressSanitizer and UndefinedBehaviorSanitizer (host code
only), so an out-of-bounds access or undefined operation in the eigensolver
fails the run."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = r"""
#include <cstdio>
#include "herm_eig.h"
int main() {
  int n;
  if (std::scanf("%d", &n) != 1) return 1;
  std::vector<std::complex<double>> A((size_t)n * n);
  for (auto& x : A) { double re, im; if (std::scanf("%lf %lf", &re, &im) != 2) return 1; x = {re, im}; }
  std::vector<double> w; std::vector<std::complex<double>> V;
  lgw::herm_eig(n, A.data(), w, V);
  for (double x : w) std::printf("%.17g\n", x);
  for (auto& x : V) std::printf("%.17g %.17g\n", x.real(), x.imag());
  return 0;
}
"""


SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module", params=["plain", "sanitized"])
def driver(request, tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("eig")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    flags = SANITIZE if request.param == "sanitized" else []
    r = subprocess.run([gxx, "-O2", "-g", "-std=c++17", *flags, "-I",
                        os.path.join(ROOT, "paper_1408_3036_amd", "csrc"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    if r.returncode != 0:
        if request.param == "sanitized":
            pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
        raise RuntimeError(r.stderr)
    return str(exe)


def _eig(exe, A):
    n = A.shape[0]
    inp = f"{n}\n" + "\n".join(f"{float(x.real)!r} {float(x.imag)!r}" for x in A.ravel()) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    w = np.array([float(x) for x in out[:n]])
    V = np.array([complex(*map(float, l.split())) for l in out[n:n + n * n]]).reshape(n, n)
    return w, V


def _herm(rng, n):
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return 0.5 * (X + X.conj().T)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 31, 64])
def test_random_hermitian(driver, n):
    A = _herm(np.random.default_rng(n), n)
    w, V = _eig(driver, A)
    assert np.abs(w - np.linalg.eigvalsh(A)).max() < 1e-12 * max(1.0, np.abs(w).max())
    assert np.abs(V.conj().T @ V - np.eye(n)).max() < 1e-12
    assert np.abs(A @ V - V * w).max() < 1e-11 * max(1.0, np.abs(w).max())


def test_degenerate_and_special(driver):
    rng = np.random.default_rng(7)
    U, _ = np.linalg.qr(rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12)))
    lam = np.array([1.0] * 4 + [-2.0] * 3 + [0.0] * 2 + [5.0, 5.0 + 1e-9, 7.0])
    A = (U * lam) @ U.conj().T
    A = 0.5 * (A + A.conj().T)
    for M in (A, np.diag(np.arange(5.0)).astype(complex), np.zeros((4, 4), complex),
              np.diag([1.0, 2.0, 3.0]) + np.diag([1.0, 1.0], 1) + np.diag([1.0, 1.0], -1)):
        w, V = _eig(driver, M)
        n = M.shape[0]
        assert np.abs(w - np.linalg.eigvalsh(M)).max() < 1e-12 * max(1.0, np.abs(w).max())
        assert np.abs(V.conj().T @ V - np.eye(n)).max() < 1e-12
        assert np.abs(M @ V - V * w).max() < 1e-11 * max(1.0, np.abs(w).max())
