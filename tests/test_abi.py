"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and argument validation fails before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1408_3036_amd import load_library
    try:
        return load_library()
    except ImportError as e:
        pytest.skip(str(e))


def test_library_exports_every_declared_symbol():
    lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "lgw.h")).read()
    names = set(re.findall(r"\b(lgw_[a-z0-9_]+)\s*\(", hdr))
    assert {"lgw_setup", "lgw_chi0_apply", "lgw_lanczos", "lgw_project"} <= names
    for n in sorted(names):
        assert hasattr(lib, n), n


def _setup(lib, **kw):
    from paper_1408_3036_amd.lgw import Opts
    N = kw.get("N", 16)
    cell = (C.c_double * 9)(*kw.get("cell", [10.0, 0, 0, 0, 10.0, 0, 0, 0, 10.0]))
    grid = (C.c_int * 3)(*kw.get("grid", [N, N, N]))
    n_v = kw.get("n_v", 2)
    V = np.zeros(N ** 3)
    psi = np.zeros((max(n_v, 1), N ** 3), dtype=np.complex128)
    eps = (C.c_double * max(n_v, 1))(*kw.get("eps", [-1.0, -0.5][:max(n_v, 1)]))
    opts = Opts()
    lib.lgw_default_opts(C.byref(opts))
    opts.mem = 1  # host memory: all validation is on the host
    for k, v in kw.get("opts", {}).items():
        setattr(opts, k, v)
    ctx = C.c_void_p()
    st = lib.lgw_setup(C.byref(ctx), cell, grid, kw.get("ecut", 6.0), V.ctypes.data, n_v,
                       psi.ctypes.data, eps, C.byref(opts))
    return st, ctx


@pytest.mark.parametrize("kw,msg", [
    (dict(grid=[16, 16, 24]), "cubic"),
    (dict(N=28), "grid N"),
    (dict(cell=[10.0, 1.0, 0, 0, 10.0, 0, 0, 0, 10.0]), "orthorhombic"),
    (dict(ecut=60.0), "does not fit"),
    (dict(ecut=-1.0), "ecut"),
    (dict(n_v=0), "n_v"),
    (dict(n_v=40), "n_v"),
    (dict(eps=[-0.5, -1.0]), "ascending"),
    (dict(opts={"tol": 0.0}), "solver options"),
    (dict(opts={"precond": 2}), "precond"),
    (dict(opts={"precond": 1, "precond_shift": 0.0}), "precond_shift"),
    (dict(opts={"imag_form": 3}), "imag_form"),
    (dict(opts={"multishift": 2}), "multishift"),
    (dict(opts={"model": 2}), "model"),
])
def test_setup_rejects_invalid_arguments_on_the_host(kw, msg):
    lib = _lib()
    st, ctx = _setup(lib, **kw)
    assert st == 1 and not ctx.value
    assert msg in lib.lgw_last_error(None).decode()


def test_setup_rejects_non_finite_input_on_the_host():
    lib = _lib()
    st, ctx = _setup(lib, eps=[-1.0, float("nan")])
    assert st == 4 and not ctx.value


def test_calls_on_null_context_fail_cleanly():
    lib = _lib()
    assert lib.lgw_chi0_apply(None, 1, None, 1, None, None) == 1
    assert lib.lgw_lanczos(None, None, 1, None, None, None, None) == 1
    assert lib.lgw_lanczos_loss_vjp(None, None, 1, 1, None, None, None, None) == 1
    assert lib.lgw_chi0_apply_vjp(None, 1, None, 1, None, None, None, None) == 1
    assert lib.lgw_project(None, 1, None, 1, None, None) == 1
    assert lib.lgw_eps_inverse(None, 1, 1, None, None) == 1
    assert lib.lgw_ritz_values(None, 1, None, None, None) == 1
    assert lib.lgw_lanczos_resume(None, 1, 2, None, None, None, None) == 1
    assert lib.lgw_lanczos_recycle(None, None, 1, 1, None, None, None, None, None, None) == 1
    lib.lgw_free(None)
