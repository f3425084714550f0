"""ctypes binding of liblgw.so.

Argument marshalling only: torch tensors supply device memory, every step of
the computation runs in the library's HIP kernels.  There is no fallback: if
the library is missing or cannot load, this module raises.

Before each call the calling thread's current torch stream (which wrote the
inputs) is synchronised, not the whole device: other contexts may be solving
on their own streams in other threads, and a device-wide synchronisation
would break their graph captures.  The library's calls return after their
own stream has finished, so the outputs are ready for any stream.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

STATUS = {0: "LGW_OK", 1: "LGW_EINVAL", 2: "LGW_ENOMEM", 3: "LGW_EDEVICE", 4: "LGW_ENAN",
          5: "LGW_ENOCONV", 6: "LGW_EBREAKDOWN"}
FLAG_CONV, FLAG_BREAK, FLAG_MAXIT = 1, 2, 4

KERNELS = {"plane_hv": 0, "zinv": 1, "zfwd": 2, "proj": 3, "cg": 4, "sqmr": 5}


class LgwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class c128(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int), ("tol", C.c_double), ("max_iter", C.c_int),
                ("check_every", C.c_int), ("precond", C.c_int), ("deterministic", C.c_int),
                ("mem", C.c_int), ("stream", C.c_void_p), ("mem_budget_gb", C.c_double),
                ("inner_tol", C.c_double), ("max_sweeps", C.c_int), ("use_graph", C.c_int),
                ("precond_shift", C.c_double), ("imag_form", C.c_int), ("multishift", C.c_int),
                ("model", C.c_int), ("autotune", C.c_int)]


class Info(C.Structure):
    _fields_ = [("N", C.c_int), ("npw", C.c_int), ("ncols", C.c_int), ("n_v", C.c_int),
                ("omega", C.c_double)]


class Timing(C.Structure):
    _fields_ = [("launches", C.c_longlong), ("total_ms", C.c_double), ("model_bytes", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("n_solves", C.c_int), ("iters", C.POINTER(C.c_int)),
                ("rel_resid", C.POINTER(C.c_double)), ("refine_sweeps", C.POINTER(C.c_int)),
                ("flags", C.POINTER(C.c_int)), ("total_iters", C.c_longlong),
                ("total_happly", C.c_longlong)]


def library_path() -> str:
    return os.environ.get("LGW_LIBRARY", os.path.join(HERE, "liblgw.so"))


_lib = None


def load_library():
    """Load liblgw.so and declare its signatures; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run `python -m paper_1408_3036_amd.build`")
    lib = C.CDLL(path)
    P, I, D = C.c_void_p, C.c_int, C.c_double
    lib.lgw_default_opts.argtypes = [C.POINTER(Opts)]
    lib.lgw_default_opts.restype = None
    lib.lgw_setup.argtypes = [C.POINTER(P), C.POINTER(D), C.POINTER(I), D, P, I, P,
                              C.POINTER(D), C.POINTER(Opts)]
    lib.lgw_chi0_apply.argtypes = [P, I, P, I, C.POINTER(c128), P]
    lib.lgw_lanczos.argtypes = [P, P, I, P, P, P, C.POINTER(I)]
    lib.lgw_lanczos_project.argtypes = [P, P, I, I, C.POINTER(c128), P, P, P, P, C.POINTER(I)]
    lib.lgw_lanczos_recycle.argtypes = [P, P, I, I, C.POINTER(C.c_double), P, P, P, P, C.POINTER(I)]
    lib.lgw_project.argtypes = [P, I, P, I, C.POINTER(c128), P]
    lib.lgw_block_lanczos.argtypes = [P, I, P, I, P, P, P, C.POINTER(I)]
    lib.lgw_chi0_apply_vjp.argtypes = [P, I, P, I, C.POINTER(c128), P, P, P]
    lib.lgw_lanczos_loss_vjp.argtypes = [P, P, I, I, C.POINTER(c128), P, P, C.POINTER(I)]
    lib.lgw_chi0_apply_many.argtypes = [I, C.POINTER(P), C.POINTER(I), C.POINTER(P), I,
                                        C.POINTER(c128), C.POINTER(P)]
    lib.lgw_hpsi.argtypes = [P, I, c128, P, P]
    lib.lgw_hpsi_noalloc.argtypes = [P, I, c128, P, P]
    lib.lgw_sigma_traces.argtypes = [P, I, C.c_double, C.c_double, I, P, I, P, P, P, P]
    lib.lgw_sigma_residues.argtypes = [P, I, C.c_double, I, P, P]
    lib.lgw_tune_info.argtypes = [P, I, I, P, P, P, P]
    lib.lgw_eps_inverse.argtypes = [P, I, I, P, P]
    lib.lgw_lanczos_resume.argtypes = [P, I, I, P, P, P, P]
    lib.lgw_ritz_values.argtypes = [P, I, P, P, P]
    lib.lgw_vhalf.argtypes = [P, I, P, P]
    lib.lgw_get_info.argtypes = [P, C.POINTER(Info)]
    lib.lgw_sphere.argtypes = [P, C.POINTER(I)]
    lib.lgw_get_stats.argtypes = [P, C.POINTER(Stats)]
    lib.lgw_profile.argtypes = [P, I]
    lib.lgw_kernel_timing.argtypes = [P, I, C.POINTER(Timing)]
    lib.lgw_last_error.argtypes = [P]
    lib.lgw_last_error.restype = C.c_char_p
    lib.lgw_free.argtypes = [P]
    lib.lgw_free.restype = None
    for name in ["lgw_setup", "lgw_chi0_apply", "lgw_lanczos", "lgw_project", "lgw_block_lanczos",
                 "lgw_chi0_apply_many", "lgw_chi0_apply_vjp", "lgw_hpsi", "lgw_hpsi_noalloc",
                 "lgw_sigma_traces", "lgw_sigma_residues", "lgw_tune_info", "lgw_eps_inverse",
                 "lgw_ritz_values", "lgw_lanczos_resume",
                 "lgw_vhalf", "lgw_get_info", "lgw_sphere", "lgw_get_stats", "lgw_profile",
                 "lgw_kernel_timing"]:
        getattr(lib, name).restype = I
    _lib = lib
    return lib


def _z(zs) -> tuple:
    zs = np.atleast_1d(np.asarray(zs, dtype=np.complex128))
    arr = (c128 * len(zs))(*[c128(float(z.real), float(z.imag)) for z in zs])
    return arr, len(zs)


class Lgw:
    """One system (H, valence set) on the current HIP device.

    V: real [N, N, N] float64 CUDA tensor; psi: [n_v, N^3] complex128 CUDA
    tensor; eps: n_v floats; cell: box edges (Lx, Ly, Lz) in bohr.  Solver
    options left as None keep the library defaults; precond=True turns on the
    diagonal kinetic preconditioner and imag_form="shifted" solves the
    imaginary axis as two shifted SQMR systems instead of the squared form;
    multishift=True solves all frequencies of a call from one Lanczos recursion
    per (column, band); model=True works on the model dielectric operator
    (H -> T in the Sternheimer equations).
    """

    def __init__(self, L, N: int, ecut: float, V, psi, eps, precision: str = "fp64",
                 tol: float | None = None, max_iter: int | None = None,
                 check_every: int | None = None, mem_budget_gb: float | None = None,
                 inner_tol: float | None = None, max_sweeps: int | None = None,
                 use_graph: bool | None = None, precond: bool | None = None,
                 precond_shift: float | None = None, imag_form: str | None = None,
                 multishift: bool | None = None, model: bool | None = None,
                 autotune: bool | None = None):
        import torch
        self.torch = torch
        self.lib = load_library()
        Ls = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
        cell = (C.c_double * 9)(*np.diag(Ls).ravel().tolist())
        grid = (C.c_int * 3)(N, N, N)
        opts = Opts()
        self.lib.lgw_default_opts(C.byref(opts))
        opts.precision = {"fp64": 0, "mixed": 1}[precision]
        if tol is not None:
            opts.tol = tol
        if max_iter is not None:
            opts.max_iter = max_iter
        if check_every is not None:
            opts.check_every = check_every
        if mem_budget_gb is not None:
            opts.mem_budget_gb = mem_budget_gb
        if inner_tol is not None:
            opts.inner_tol = inner_tol
        if max_sweeps is not None:
            opts.max_sweeps = max_sweeps
        if use_graph is not None:
            opts.use_graph = int(use_graph)
        if precond is not None:
            opts.precond = int(precond)
        if precond_shift is not None:
            opts.precond_shift = precond_shift
        if imag_form is not None:
            opts.imag_form = {"squared": 0, "shifted": 1}[imag_form]
        if multishift is not None:
            opts.multishift = int(multishift)
        if model is not None:
            opts.model = int(model)
        if autotune is not None:
            opts.autotune = int(autotune)
        self.opts = opts
        V = self._dev(V, torch.float64).reshape(-1)
        psi = self._dev(psi, torch.complex128).reshape(len(eps), -1)
        eps_arr = (C.c_double * len(eps))(*[float(e) for e in eps])
        ctx = C.c_void_p()
        torch.cuda.current_stream().synchronize()
        st = self.lib.lgw_setup(C.byref(ctx), cell, grid, float(ecut), V.data_ptr(), len(eps),
                                psi.data_ptr(), eps_arr, C.byref(opts))
        if st != 0:
            raise LgwError(st, self.lib.lgw_last_error(None).decode())
        self.ctx = ctx
        self.N = N
        self.n_v = len(eps)
        info = Info()
        self.lib.lgw_get_info(ctx, C.byref(info))
        self.npw, self.ncols, self.omega = info.npw, info.ncols, info.omega

    def _dev(self, x, dtype):
        t = self.torch
        if not isinstance(x, t.Tensor):
            x = t.as_tensor(np.asarray(x))
        return x.to(device="cuda", dtype=dtype).contiguous()

    def _check(self, st: int, allow_partial: bool = False):
        if st != 0 and not (allow_partial and st in (5, 6)):
            raise LgwError(st, self.lib.lgw_last_error(self.ctx).decode())
        return STATUS[st]

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.lgw_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- calls
    def chi0_apply(self, dV, z, allow_partial: bool = False):
        """dn[z, j] = chi0(z) dV[j]; dV [n_rhs, N^3] complex128 (CUDA)."""
        t = self.torch
        dV = self._dev(dV, t.complex128)
        dV = dV.reshape(-1, self.N ** 3)
        zarr, nz = _z(z)
        out = t.empty((nz, dV.shape[0], self.N ** 3), dtype=t.complex128, device="cuda")
        t.cuda.current_stream().synchronize()
        self.last_status = self._check(
            self.lib.lgw_chi0_apply(self.ctx, dV.shape[0], dV.data_ptr(), nz, zarr, out.data_ptr()),
            allow_partial)
        return out

    def chi0_apply_vjp(self, dV, z, g_dn, want_dV: bool = True, want_V: bool = True):
        """Gradients of L = Re sum conj(g_dn) * chi0_apply(dV, z):
        returns (dL/d dV as a complex tensor [n_rhs, N^3] or None,
                 dL/dV_loc as a float64 tensor [N^3] or None)."""
        t = self.torch
        dV = self._dev(dV, t.complex128).reshape(-1, self.N ** 3)
        zarr, nz = _z(z)
        g = self._dev(g_dn, t.complex128).reshape(nz, dV.shape[0], self.N ** 3)
        gdV = t.empty_like(dV) if want_dV else None
        gV = t.empty(self.N ** 3, dtype=t.float64, device="cuda") if want_V else None
        t.cuda.current_stream().synchronize()
        self.last_status = self._check(self.lib.lgw_chi0_apply_vjp(
            self.ctx, dV.shape[0], dV.data_ptr(), nz, zarr, g.data_ptr(),
            gdV.data_ptr() if gdV is not None else None, gV.data_ptr() if gV is not None else None))
        return gdV, gV

    def lanczos(self, q0, k: int, want_Q: bool = True):
        t = self.torch
        q0 = self._dev(q0, t.complex128).reshape(-1)
        alpha = t.zeros(k, dtype=t.float64, device="cuda")
        beta = t.zeros(k, dtype=t.float64, device="cuda")
        Q = t.zeros((k, self.N ** 3), dtype=t.complex128, device="cuda") if want_Q else None
        kd = C.c_int(0)
        t.cuda.current_stream().synchronize()
        self.last_status = self._check(self.lib.lgw_lanczos(
            self.ctx, q0.data_ptr(), k, alpha.data_ptr(), beta.data_ptr(),
            Q.data_ptr() if Q is not None else None, C.byref(kd)))
        n = kd.value
        return alpha[:n], beta[:n], (Q[:n] if Q is not None else None), n

    def lanczos_resume(self, alpha, beta, Q, k: int):
        """Continue a recursion from its first k0 = len(alpha) steps (alpha,
        beta [k0], Q [k0, N^3]) to k steps (lgw_lanczos_resume)."""
        t = self.torch
        k0 = int(alpha.shape[0])
        a = t.zeros(k, dtype=t.float64, device="cuda")
        b = t.zeros(k, dtype=t.float64, device="cuda")
        Qo = t.zeros((k, self.N ** 3), dtype=t.complex128, device="cuda")
        a[:k0] = self._dev(alpha, t.float64)
        b[:k0] = self._dev(beta, t.float64)
        Qo[:k0] = self._dev(Q, t.complex128).reshape(k0, -1)
        kd = C.c_int(0)
        t.cuda.current_stream().synchronize()
        self.last_status = self._check(self.lib.lgw_lanczos_resume(
            self.ctx, k0, k, a.data_ptr(), b.data_ptr(), Qo.data_ptr(), C.byref(kd)))
        n = kd.value
        return a[:n], b[:n], Qo[:n], n

    def lanczos_loss_vjp(self, q0, k: int, z, want_V: bool = True):
        """L = sum_z log det(I + Q^H (eps(z)-1) Q) with Q the k-step Lanczos
        basis of eps(0)-1 from q0, and dL/dV_loc (float64 [N^3], or None).
        Returns (L, gradient, number of Lanczos vectors used)."""
        t = self.torch
        q0 = self._dev(q0, t.complex128).reshape(-1)
        zarr, nz = _z(z)
        loss = t.zeros(1, dtype=t.float64, device="cuda")
        gV = t.empty(self.N ** 3, dtype=t.float64, device="cuda") if want_V else None
        kd = C.c_int(0)
        t.cuda.current_stream().synchronize()
        self.last_status = self._check(self.lib.lgw_lanczos_loss_vjp(
            self.ctx, q0.data_ptr(), k, nz, zarr, loss.data_ptr(),
            gV.data_ptr() if gV is not None else None, C.byref(kd)))
        return float(loss.item()), gV, kd.value

    def lanczos_project(self, q0, k: int, z, want_Q: bool = True):
        """lanczos(q0, k) and project(Q, z) in one call, the projection of
        finished Lanczos vectors overlapped with the recursion.  Returns
        (alpha, beta, Q, E [n_z, k_done, k_done], k_done)."""
        t = self.torch
        q0 = self._dev(q0, t.complex128).reshape(-1)
        zarr, nz = _z(z)
        alpha = t.zeros(k, dtype=t.float64, device="cuda")
        beta = t.zeros(k, dtype=t.float64, device="cuda")
        Q = t.zeros((k, self.N ** 3), dtype=t.complex128, device="cuda") if want_Q else None
        E = t.zeros((nz, k, k), dtype=t.complex128, device="cuda")
        kd = C.c_int(0)
        t.cuda.current_stream().synchronize()
        self.last_status = self._check(self.lib.lgw_lanczos_project(
            self.ctx, q0.data_ptr(), k, nz, zarr, alpha.data_ptr(), beta.data_ptr(),
            Q.data_ptr() if Q is not None else None, E.data_ptr(), C.byref(kd)))
        n = kd.value
        return alpha[:n], beta[:n], (Q[:n] if Q is not None else None), E[:, :n, :n], n

    def lanczos_recycle(self, q0, k: int, w, want_Q: bool = True):
        """lanczos(q0, k) and eps(i w) - 1 on its vectors at the imaginary
        frequencies i*w by frequency recycling (one small basis per band).
        Returns (alpha, beta, Q, E [n_w, k_done, k_done], k_done)."""
        t = self.torch
        q0 = self._dev(q0, t.complex128).reshape(-1)
        wl = [float(x) for x in w]
        warr = (C.c_double * len(wl))(*wl)
        alpha = t.zeros(k, dtype=t.float64, device="cuda")
        beta = t.zeros(k, dtype=t.float64, device="cuda")
        Q = t.zeros((k, self.N ** 3), dtype=t.complex128, device="cuda") if want_Q else None
        E = t.zeros((len(wl), k, k), dtype=t.complex128, device="cuda")
        kd = C.c_int(0)
        t.cuda.current_stream().synchronize()
        self.last_status = self._check(self.lib.lgw_lanczos_recycle(
            self.ctx, q0.data_ptr(), k, len(wl), warr, alpha.data_ptr(), beta.data_ptr(),
            Q.data_ptr() if Q is not None else None, E.data_ptr(), C.byref(kd)))
        n = kd.value
        return alpha[:n], beta[:n], (Q[:n] if Q is not None else None), E[:, :n, :n], n

    def block_lanczos(self, Q0, nblk: int, want_Q: bool = True):
        """Block Lanczos from the rows of Q0 [b, N^3]: returns A, B [nblk, b, b], Q, nblk_done."""
        t = self.torch
        Q0 = self._dev(Q0, t.complex128).reshape(-1, self.N ** 3)
        b = Q0.shape[0]
        A = t.zeros((nblk, b, b), dtype=t.complex128, device="cuda")
        B = t.zeros((nblk, b, b), dtype=t.complex128, device="cuda")
        Q = t.zeros((nblk * b, self.N ** 3), dtype=t.complex128, device="cuda") if want_Q else None
        nd = C.c_int(0)
        t.cuda.current_stream().synchronize()
        self.last_status = self._check(self.lib.lgw_block_lanczos(
            self.ctx, b, Q0.data_ptr(), nblk, A.data_ptr(), B.data_ptr(),
            Q.data_ptr() if Q is not None else None, C.byref(nd)))
        n = nd.value
        return A[:n], B[:n], (Q[:n * b] if Q is not None else None), n

    def project(self, Q, z):
        t = self.torch
        Q = self._dev(Q, t.complex128)
        k = Q.shape[0]
        zarr, nz = _z(z)
        E = t.empty((nz, k, k), dtype=t.complex128, device="cuda")
        t.cuda.current_stream().synchronize()
        self.last_status = self._check(
            self.lib.lgw_project(self.ctx, k, Q.data_ptr(), nz, zarr, E.data_ptr()))
        return E

    def eps_inverse(self, E):
        """(I + E[z])^-1 for E [n_z, k, k] complex128 (lgw_eps_inverse)."""
        t = self.torch
        E = self._dev(E, t.complex128)
        if E.dim() == 2:
            E = E[None]
        nz, k = E.shape[0], E.shape[1]
        out = t.empty_like(E)
        t.cuda.current_stream().synchronize()
        self._check(self.lib.lgw_eps_inverse(self.ctx, k, nz, E.data_ptr(), out.data_ptr()))
        return out

    def ritz_values(self, alpha, beta):
        """Eigenvalues of the Lanczos tridiagonal (lgw_ritz_values), ascending."""
        t = self.torch
        alpha = self._dev(alpha, t.float64).reshape(-1)
        k = alpha.shape[0]
        beta = self._dev(beta, t.float64).reshape(-1) if k > 1 else None
        theta = np.zeros(k)
        t.cuda.current_stream().synchronize()
        self._check(self.lib.lgw_ritz_values(self.ctx, k, alpha.data_ptr(),
                                             beta.data_ptr() if beta is not None else None, theta.ctypes.data))
        return theta

    def hpsi(self, x, shift: complex = 0.0):
        t = self.torch
        x = self._dev(x, t.complex128).reshape(-1, self.npw)
        y = t.empty_like(x)
        t.cuda.current_stream().synchronize()
        self._check(self.lib.lgw_hpsi(self.ctx, x.shape[0], c128(shift.real, shift.imag),
                                      x.data_ptr(), y.data_ptr()))
        return y

    def sigma_traces(self, e: int, delta: float, Q, w, alpha: float = 1.0):
        """Self-energy integrand traces in the basis Q [k, N^3] (lgw_sigma_traces):
        returns (sigma_N [n_w], sigma_N0 [n_w], sigma_A)."""
        t = self.torch
        Q = self._dev(Q, t.complex128).reshape(-1, self.N ** 3)
        w = np.ascontiguousarray(np.atleast_1d(np.asarray(w, dtype=np.float64)))
        sN = np.zeros(len(w))
        sN0 = np.zeros(len(w))
        sA = np.zeros(1)
        t.cuda.current_stream().synchronize()
        self.last_status = self._check(self.lib.lgw_sigma_traces(
            self.ctx, int(e), float(delta), float(alpha), Q.shape[0], Q.data_ptr(), len(w),
            w.ctypes.data, sN.ctypes.data, sN0.ctypes.data, sA.ctypes.data))
        return sN, sN0, float(sA[0])

    def tune_info(self, precision: str, nsys: int) -> dict:
        """Plane-pass tile variant used for nsys systems (lgw_tune_info)."""
        v, nt, pd = C.c_int(0), C.c_int(0), C.c_int(0)
        us = (C.c_double * 4)()
        self._check(self.lib.lgw_tune_info(self.ctx, {"fp64": 0, "mixed": 1}[precision], int(nsys),
                                           C.byref(v), C.byref(nt), C.byref(pd), us))
        return {"variant": v.value, "threads": nt.value, "padded_rows": pd.value, "us": list(us)}

    def sigma_residues(self, e: int, delta: float, k_p: int = 4):
        """Residue term Sigma_P of state e (lgw_sigma_residues): (Sigma_P, n_poles)."""
        sp = np.zeros(1)
        npl = C.c_int(0)
        self.torch.cuda.current_stream().synchronize()
        self.last_status = self._check(self.lib.lgw_sigma_residues(
            self.ctx, int(e), float(delta), int(k_p), sp.ctypes.data, C.byref(npl)))
        return float(sp[0]), npl.value

    def hpsi_noalloc(self, x, y, shift: complex = 0.0):
        """y = (H - shift) x into the caller's device tensor y through
        lgw_hpsi_noalloc (no allocation in the library; asynchronous on the
        context's stream: synchronise before reading y)."""
        t = self.torch
        assert x.is_cuda and y.is_cuda and x.dtype == t.complex128 and y.dtype == t.complex128
        assert x.is_contiguous() and y.is_contiguous() and x.shape == y.shape and x.shape[-1] == self.npw
        n = x.numel() // self.npw
        self._check(self.lib.lgw_hpsi_noalloc(self.ctx, n, c128(shift.real, shift.imag),
                                              x.data_ptr(), y.data_ptr()))
        return y

    def vhalf(self, x):
        t = self.torch
        x = self._dev(x, t.complex128).reshape(-1, self.N ** 3)
        y = t.empty_like(x)
        t.cuda.current_stream().synchronize()
        self._check(self.lib.lgw_vhalf(self.ctx, x.shape[0], x.data_ptr(), y.data_ptr()))
        return y

    def sphere(self) -> np.ndarray:
        m = (C.c_int * (3 * self.npw))()
        self._check(self.lib.lgw_sphere(self.ctx, m))
        return np.frombuffer(m, dtype=np.int32).reshape(self.npw, 3).copy()

    def profile(self, enable: bool = True):
        """Turn per-kernel HIP-event timing on/off (resets the counters)."""
        self._check(self.lib.lgw_profile(self.ctx, int(enable)))

    def kernel_timing(self) -> dict:
        """{'<kernel>_f64' / '<kernel>_f32': launches, total_ms, model_bytes}."""
        out = {}
        for name, k in KERNELS.items():
            for suf, off in (("f64", 0), ("f32", 8)):
                t = Timing()
                self._check(self.lib.lgw_kernel_timing(self.ctx, k + off, C.byref(t)))
                if t.launches:
                    out[f"{name}_{suf}"] = {"launches": t.launches, "total_ms": t.total_ms,
                                            "model_bytes": t.model_bytes}
        return out

    def stats(self) -> dict:
        s = Stats()
        self._check(self.lib.lgw_get_stats(self.ctx, C.byref(s)))
        n = s.n_solves

        def arr(p, dt):
            return np.ctypeslib.as_array(p, shape=(n,)).astype(dt).copy() if n else np.zeros(0, dt)
        return {"n_solves": n, "iters": arr(s.iters, np.int64),
                "rel_resid": arr(s.rel_resid, np.float64),
                "refine_sweeps": arr(s.refine_sweeps, np.int64),
                "flags": arr(s.flags, np.int64), "total_iters": s.total_iters,
                "total_happly": s.total_happly}


def chi0_apply_many(systems, dVs, z, allow_partial: bool = False):
    """chi0(z) on several independent systems in one call (uneven sizes allowed).

    systems: list of Lgw; dVs: list of [n_rhs_i, N_i^3] complex128 tensors.
    Returns a list of [n_z, n_rhs_i, N_i^3] tensors.
    """
    import torch
    lib = load_library()
    n = len(systems)
    dVs = [s._dev(d, torch.complex128).reshape(-1, s.N ** 3) for s, d in zip(systems, dVs)]
    zarr, nz = _z(z)
    outs = [torch.empty((nz, d.shape[0], s.N ** 3), dtype=torch.complex128, device="cuda")
            for s, d in zip(systems, dVs)]
    ctxs = (C.c_void_p * n)(*[s.ctx.value for s in systems])
    nr = (C.c_int * n)(*[d.shape[0] for d in dVs])
    ins = (C.c_void_p * n)(*[d.data_ptr() for d in dVs])
    ous = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
    torch.cuda.current_stream().synchronize()
    st = lib.lgw_chi0_apply_many(n, ctxs, nr, ins, nz, zarr, ous)
    if st != 0 and not (allow_partial and st in (5, 6)):
        raise LgwError(st, "lgw_chi0_apply_many failed")
    return outs

