"""Python binding of libnosdd (ctypes).  Argument marshalling only: every step
of the solve runs in the library's HIP kernels; PyTorch supplies device memory
and the stream.  The library must be built (``python -m
paper_2509_03622_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libnosdd.so")

OK, NOT_CONVERGED = 0, 1
STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EPARTITION",
          -5: "EBREAKDOWN", -6: "ENONFINITE", -7: "ENOWEIGHTS", -8: "ESTATE"}

EXPORTS = ["nosdd_ctx_create", "nosdd_ctx_destroy", "nosdd_last_error", "nosdd_problem_create",
           "nosdd_problem_create_cores",
           "nosdd_problem_setup", "nosdd_problem_destroy", "nosdd_solve", "nosdd_solve_device", "nosdd_solve_device_c64", "nosdd_solve_paper_device",
           "nosdd_apply_operator", "nosdd_schwarz_sweep", "nosdd_precond_apply", "nosdd_local_solve",
           "nosdd_robin_trace", "nosdd_tile_info", "nosdd_sizes", "nosdd_last_timing", "nosdd_coarse_basis",
           "nosdd_profile", "nosdd_kernel_times", "nosdd_nn_apply", "nosdd_graphs", "nosdd_multi_source", "nosdd_stored_basis", "nosdd_autotune", "nosdd_tuning",
           "nosdd_fom_gradient_device", "nosdd_fallback_count", "nosdd_precond_apply_noalloc"]


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("h", C.c_double), ("npml", C.c_int),
                ("pml_m", C.c_int), ("pml_lnR", C.c_double)]


class PartitionSpec(C.Structure):
    _fields_ = [("core_x", C.POINTER(C.c_int)), ("ncx", C.c_int), ("core_y", C.POINTER(C.c_int)),
                ("ncy", C.c_int), ("overlap", C.c_int)]


class SetupOpts(C.Structure):
    _fields_ = [("sub_solver", C.c_int), ("k_coarse", C.c_int), ("k_trial", C.c_int),
                ("nn_weights", C.c_char_p), ("inner_max", C.c_int), ("inner_tol", C.c_float)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int), ("max_iters", C.c_int), ("x0", C.c_void_p)]


class PaperOpts(C.Structure):
    _fields_ = [("momentum", C.c_double), ("coarse", C.c_int), ("tol", C.c_double), ("max_iters", C.c_int)]


class NosddError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path=LIBPATH):
    """Load libnosdd.so and declare its C signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2509_03622_amd.build`")
    try:
        # torch brings its own HIP runtime; loading it first makes the library
        # bind to that one, so torch's streams and memory are valid in both
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(path)
    vp, i, ll = C.c_void_p, C.c_int, C.c_longlong
    sig = {
        "nosdd_ctx_create": (i, [i, vp, C.POINTER(vp)]),
        "nosdd_ctx_destroy": (None, [vp]),
        "nosdd_last_error": (C.c_char_p, [vp]),
        "nosdd_problem_create": (i, [vp, C.POINTER(Grid), vp, C.POINTER(PartitionSpec), vp, i, C.POINTER(vp)]),
        "nosdd_problem_create_cores": (i, [vp, C.POINTER(Grid), vp, vp, i, i, vp, i, C.POINTER(vp)]),
        "nosdd_problem_setup": (i, [vp, C.POINTER(SetupOpts)]),
        "nosdd_problem_destroy": (None, [vp]),
        "nosdd_solve": (i, [vp, vp, i, C.POINTER(SolveOpts), vp, vp, vp, vp]),
        "nosdd_solve_device": (i, [vp, vp, i, C.POINTER(SolveOpts), vp, vp, vp, vp]),
        "nosdd_solve_paper_device": (i, [vp, vp, i, C.POINTER(PaperOpts), vp, vp, vp, vp]),
        "nosdd_solve_device_c64": (i, [vp, vp, i, C.POINTER(SolveOpts), vp, vp, vp, vp]),
        "nosdd_apply_operator": (i, [vp, vp, vp, vp, i]),
        "nosdd_schwarz_sweep": (i, [vp, vp, vp, i]),
        "nosdd_precond_apply": (i, [vp, vp, vp, vp, i]),
        "nosdd_local_solve": (i, [vp, vp, vp]),
        "nosdd_robin_trace": (i, [vp, vp, vp]),
        "nosdd_tile_info": (i, [vp, i, C.POINTER(ll)]),
        "nosdd_sizes": (i, [vp, C.POINTER(i), C.POINTER(ll), C.POINTER(ll), C.POINTER(i)]),
        "nosdd_last_timing": (i, [vp, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(i)]),
        "nosdd_coarse_basis": (i, [vp, i, vp, vp]),
        "nosdd_profile": (i, [vp, i]),
        "nosdd_kernel_times": (i, [vp, vp, vp, vp]),
        "nosdd_nn_apply": (i, [vp, vp, vp]),
        "nosdd_graphs": (i, [vp, i]),
        "nosdd_multi_source": (i, [vp, i]),
        "nosdd_stored_basis": (i, [vp, i]),
        "nosdd_autotune": (i, [vp, i]),
        "nosdd_tuning": (i, [vp, vp]),
        "nosdd_fom_gradient_device": (i, [vp, vp, i, vp, i, C.POINTER(SolveOpts), C.POINTER(C.c_double), vp, vp]),
        "nosdd_fallback_count": (i, [vp, C.POINTER(ll)]),
        "nosdd_precond_apply_noalloc": (i, [vp, vp, vp, vp, i]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _ptr(a):
    """Data pointer of a torch tensor or a numpy array (C-contiguous)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr()
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return a.ctypes.data


class Context:
    def __init__(self, device=0, stream=None):
        L = load()
        self.L = L
        h = C.c_void_p()
        st = L.nosdd_ctx_create(device, stream, C.byref(h))
        if st != OK:
            raise NosddError(st, "nosdd_ctx_create failed")
        self.h = h
        self._problems = weakref.WeakSet()

    def check(self, st):
        if st < 0:
            raise NosddError(st, self.L.nosdd_last_error(self.h).decode())
        return st

    def close(self):
        # problems live on this context: release them first, whatever order
        # the garbage collector finalises the Python objects in
        for prob in list(getattr(self, "_problems", ())):
            prob.close()
        if self.h:
            self.L.nosdd_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """A grid, permittivity map, partition and wavelength set (one operator per wavelength)."""

    def __init__(self, ctx: Context, eps, h, npml, core_x, core_y, overlap, wavelengths, pml_m=2, pml_lnR=-30.0,
                 cores=None):
        """core_x, core_y: tensor-product partition; or cores: an explicit list of
        (cx0, cx1, cy0, cy1) rectangles covering the grid (core_x, core_y ignored)."""
        self.ctx, self.L = ctx, ctx.L
        eps = np.ascontiguousarray(eps, dtype=np.float32)
        self.ny, self.nx = eps.shape
        self.wavelengths = [float(w) for w in wavelengths]
        g = Grid(self.nx, self.ny, float(h), int(npml), int(pml_m), float(pml_lnR))
        wl = np.ascontiguousarray(self.wavelengths, dtype=np.float64)
        hp = C.c_void_p()
        if cores is not None:
            cv = np.ascontiguousarray(np.asarray(cores, dtype=np.int32).reshape(-1, 4))
            ctx.check(self.L.nosdd_problem_create_cores(ctx.h, C.byref(g), eps.ctypes.data, cv.ctypes.data,
                                                        cv.shape[0], int(overlap), wl.ctypes.data, len(wl),
                                                        C.byref(hp)))
        else:
            cx = (C.c_int * len(core_x))(*core_x)
            cy = (C.c_int * len(core_y))(*core_y)
            part = PartitionSpec(cx, len(core_x), cy, len(core_y), int(overlap))
            ctx.check(self.L.nosdd_problem_create(ctx.h, C.byref(g), eps.ctypes.data, C.byref(part),
                                                  wl.ctypes.data, len(wl), C.byref(hp)))
        self.h = hp
        self.n_wl = len(wl)
        ctx._problems.add(self)

    def setup(self, k_coarse=0, k_trial=8, sub_solver=0, nn_weights=None, inner_max=2, inner_tol=1e-1):
        o = SetupOpts(sub_solver, k_coarse, k_trial, nn_weights.encode() if nn_weights else None, inner_max,
                      inner_tol)
        return self.ctx.check(self.L.nosdd_problem_setup(self.h, C.byref(o)))

    def close(self):
        if getattr(self, "h", None) and self.ctx.h:
            self.L.nosdd_problem_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ whole solves
    def solve(self, J, tol=1e-6, restart=30, max_iters=1000, x0=None):
        """Host arrays in and out.  J [n_src][ny][nx] complex64."""
        J = np.ascontiguousarray(J, dtype=np.complex64)
        if J.ndim == 2:
            J = J[None]
        ns = J.shape[0]
        nr = self.n_wl * ns
        E = np.zeros((self.n_wl, ns, self.ny, self.nx), np.complex64)
        hist = np.zeros((self.n_wl, ns, max(1, max_iters)), np.float32)
        iters = np.zeros((self.n_wl, ns), np.int32)
        fin = np.zeros((self.n_wl, ns), np.float32)
        x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.complex64)
        o = SolveOpts(tol, restart, max_iters, _ptr(x0a))
        st = self.ctx.check(self.L.nosdd_solve(self.h, J.ctypes.data, ns, C.byref(o), E.ctypes.data,
                                               hist.ctypes.data, iters.ctypes.data, fin.ctypes.data))
        del nr
        return E, hist, iters, fin, st

    def solve_device_c64(self, J, E64, tol=1e-6, restart=30, max_iters=1000, x0=None):
        """As solve_device, with E64 [n_wl][n_src][ny][nx] complex128 receiving the FP64 iterate."""
        ns = J.shape[0]
        hist = np.zeros((self.n_wl, ns, max(1, max_iters)), np.float32)
        iters = np.zeros((self.n_wl, ns), np.int32)
        fin = np.zeros((self.n_wl, ns), np.float32)
        o = SolveOpts(tol, restart, max_iters, _ptr(x0))
        st = self.ctx.check(self.L.nosdd_solve_device_c64(self.h, _ptr(J), ns, C.byref(o), _ptr(E64),
                                                          hist.ctypes.data, iters.ctypes.data, fin.ctypes.data))
        return hist, iters, fin, st

    def solve_paper(self, J, E, momentum=0.0, coarse=False, tol=1e-6, max_iters=500):
        """The paper's Algorithm 3 loop on device tensors (J [n_src][ny][nx],
        E [n_wl][n_src][ny][nx] complex64); returns (hist, sweeps, final, status)."""
        ns = J.shape[0]
        hist = np.zeros((self.n_wl, ns, max(1, max_iters)), np.float32)
        iters = np.zeros((self.n_wl, ns), np.int32)
        fin = np.zeros((self.n_wl, ns), np.float32)
        o = PaperOpts(momentum, 1 if coarse else 0, tol, max_iters)
        st = self.ctx.check(self.L.nosdd_solve_paper_device(self.h, _ptr(J), ns, C.byref(o), _ptr(E),
                                                            hist.ctypes.data, iters.ctypes.data, fin.ctypes.data))
        return hist, iters, fin, st

    def solve_device(self, J, E, tol=1e-6, restart=30, max_iters=1000, x0=None):
        """Device tensors: J [n_src][ny][nx] complex64, E [n_wl][n_src][ny][nx] complex64."""
        ns = J.shape[0]
        hist = np.zeros((self.n_wl, ns, max(1, max_iters)), np.float32)
        iters = np.zeros((self.n_wl, ns), np.int32)
        fin = np.zeros((self.n_wl, ns), np.float32)
        o = SolveOpts(tol, restart, max_iters, _ptr(x0))
        st = self.ctx.check(self.L.nosdd_solve_device(self.h, _ptr(J), ns, C.byref(o), _ptr(E), hist.ctypes.data,
                                                      iters.ctypes.data, fin.ctypes.data))
        return hist, iters, fin, st

    # ------------------------------------------------------------ sweep steps (device tensors)
    def apply_operator(self, x, y, b=None, n_src=1):
        return self.ctx.check(self.L.nosdd_apply_operator(self.h, _ptr(x), _ptr(b), _ptr(y), n_src))

    def schwarz_sweep(self, v, z, n_src=1):
        return self.ctx.check(self.L.nosdd_schwarz_sweep(self.h, _ptr(v), _ptr(z), n_src))

    def precond_apply(self, v, z, Az=None, n_src=1):
        return self.ctx.check(self.L.nosdd_precond_apply(self.h, _ptr(v), _ptr(z), _ptr(Az), n_src))

    def precond_apply_noalloc(self, v, z, Az, n_src=1):
        """Two-level preconditioner without any device allocation (fixed library scratch)."""
        return self.ctx.check(self.L.nosdd_precond_apply_noalloc(self.h, _ptr(v), _ptr(z), _ptr(Az), n_src))

    def local_solve(self, rhs, u):
        return self.ctx.check(self.L.nosdd_local_solve(self.h, _ptr(rhs), _ptr(u)))

    def nn_apply(self, v, e):
        return self.ctx.check(self.L.nosdd_nn_apply(self.h, _ptr(v), _ptr(e)))

    def robin_trace(self, x, g):
        return self.ctx.check(self.L.nosdd_robin_trace(self.h, _ptr(x), _ptr(g)))

    # ------------------------------------------------------------ queries
    def sizes(self):
        nt, nc = C.c_int(), C.c_int()
        lc, te = C.c_longlong(), C.c_longlong()
        self.ctx.check(self.L.nosdd_sizes(self.h, C.byref(nt), C.byref(lc), C.byref(te), C.byref(nc)))
        return nt.value, lc.value, te.value, nc.value

    def tile_info(self, t):
        a = (C.c_longlong * 10)()
        self.ctx.check(self.L.nosdd_tile_info(self.h, t, a))
        return list(a)

    def coarse_basis(self, wl=0):
        """Basis fields per tile: list (per tile) of arrays [k_coarse][bh][bw] and box origins."""
        nt, lc, ne, nc = self.sizes()
        box = np.zeros((nt, 4), np.int64)
        self.ctx.check(self.L.nosdd_coarse_basis(self.h, wl, None, box.ctypes.data))
        if nc == 0:
            return [], box
        kc = nc // nt
        total = int(sum(kc * b[2] * b[3] for b in box))
        phi = np.zeros(total, np.complex64)
        self.ctx.check(self.L.nosdd_coarse_basis(self.h, wl, phi.ctypes.data, None))
        out, off = [], 0
        for b in box:
            n = kc * int(b[2]) * int(b[3])
            out.append(phi[off:off + n].reshape(kc, int(b[3]), int(b[2])))
            off += n
        return out, box

    def fom_gradient(self, J, focal, tol=1e-6, restart=30, max_iters=1000):
        """FoM = sum |E(r_f)|^2 over wavelengths, sources, focal cells and its gradient
        d FoM / d eps [ny][nx] (device float32 tensor), by a forward and an adjoint solve.
        J: device complex64 [n_src][ny][nx]; focal: sequence of (ix, iy).
        Returns (fom, grad, iters [2][n_wl][n_src], status)."""
        import torch
        ns = J.shape[0]
        foc = np.ascontiguousarray(np.asarray(focal, dtype=np.int32).reshape(-1, 2))
        grad = torch.empty((self.ny, self.nx), dtype=torch.float32, device=J.device)
        iters = np.zeros((2, self.n_wl, ns), np.int32)
        fom = C.c_double(0.0)
        o = SolveOpts(tol, restart, max_iters, None)
        st = self.ctx.check(self.L.nosdd_fom_gradient_device(self.h, _ptr(J), ns, foc.ctypes.data, foc.shape[0],
                                                             C.byref(o), C.byref(fom), _ptr(grad),
                                                             iters.ctypes.data))
        return fom.value, grad, iters, st

    def autotune(self, enable=True):
        """Time candidate launch parameters at the first solve of a batch shape (default on)."""
        return self.ctx.check(self.L.nosdd_autotune(self.h, 1 if enable else 0))

    def tuning(self):
        """{depth, nblk per basis bucket, flags} chosen by the autotuner."""
        out = np.zeros(6, np.int32)
        self.ctx.check(self.L.nosdd_tuning(self.h, out.ctypes.data))
        return {"solve_prefetch_depth": int(out[0]), "gs_workgroups_per_rhs": out[1:5].tolist(),
                "tuned_gram_schmidt": bool(out[5] & 1), "tuned_subdomain_solve": bool(out[5] & 2)}

    def multi_source(self, enable=True):
        """Solve the sources of a wavelength together (one factor stream, MFMA products) or one by one."""
        return self.ctx.check(self.L.nosdd_multi_source(self.h, 1 if enable else 0))

    def stored_basis(self, enable=True):
        """Second Gram-Schmidt pass in coefficient space (two passes per step) or as a third pass."""
        return self.ctx.check(self.L.nosdd_stored_basis(self.h, 1 if enable else 0))

    def graphs(self, enable=True):
        """Replay captured per-step HIP graphs (default) or launch kernels one by one."""
        return self.ctx.check(self.L.nosdd_graphs(self.h, 1 if enable else 0))

    def profile(self, enable=True):
        return self.ctx.check(self.L.nosdd_profile(self.h, 1 if enable else 0))

    def kernel_times(self):
        """(ms[4], launches[4], units[4]) per class: local solve, operator, Arnoldi, coarse."""
        ms = np.zeros(4, np.float64)
        la = np.zeros(4, np.int64)
        un = np.zeros(4, np.int64)
        self.ctx.check(self.L.nosdd_kernel_times(self.h, ms.ctypes.data, la.ctypes.data, un.ctypes.data))
        return ms, la, un

    def fallback_count(self):
        """Inner NN-FGMRES solves replaced by the exact subdomain LU solve since the last solve began."""
        c = C.c_longlong()
        self.ctx.check(self.L.nosdd_fallback_count(self.h, C.byref(c)))
        return int(c.value)

    def last_timing(self):
        s, v, i = C.c_double(), C.c_double(), C.c_int()
        self.ctx.check(self.L.nosdd_last_timing(self.h, C.byref(s), C.byref(v), C.byref(i)))
        return s.value, v.value, i.value


def torch_stream_handle():
    """The current PyTorch HIP stream as a raw handle for Context(stream=...)."""
    import torch
    return torch.cuda.current_stream().cuda_stream


def _fom_function():
    import torch

    class FomGradient(torch.autograd.Function):
        """FoM(eps) = sum over wavelengths, sources and focal cells of |E(r_f)|^2 with
        E = A(eps)^-1 (-i omega J), differentiable in eps through the library's
        adjoint solve (the backward pass reuses the gradient computed with the FoM).
        Every call builds and factorises the problem for the given eps."""

        @staticmethod
        def forward(ctx_, eps, J, focal, spec):
            ctx = Context(0, torch_stream_handle())
            P = Problem(ctx, eps.detach().cpu().numpy().astype(np.float32), spec["h"], spec["npml"],
                        spec["core_x"], spec["core_y"], spec["overlap"], spec["wavelengths"],
                        spec.get("pml_m", 2), spec.get("pml_lnR", -30.0))
            P.setup(k_coarse=spec.get("k_coarse", 0), k_trial=spec.get("k_trial", 8))
            fom, grad, iters, st = P.fom_gradient(J, focal, tol=spec.get("tol", 1e-6),
                                                  max_iters=spec.get("max_iters", 1000))
            torch.cuda.synchronize()
            P.close()
            ctx.close()
            if st != OK:
                # a gradient from fields that did not reach tol is not the gradient of the FoM
                raise NosddError(st, "forward or adjoint solve stopped at max_iters "
                                     f"(outer iterations forward {iters[0].ravel().tolist()}, "
                                     f"adjoint {iters[1].ravel().tolist()})")
            ctx_.save_for_backward(grad.to(eps.device))
            ctx_.iters = iters
            return torch.tensor(fom, dtype=torch.float64, device=eps.device)

        @staticmethod
        def backward(ctx_, g):
            (grad,) = ctx_.saved_tensors
            return (g.to(grad.dtype) * grad, None, None, None)

    return FomGradient


def figure_of_merit(eps, J, focal, spec):
    """Differentiable FoM(eps) (see FomGradient); spec holds the grid and partition:
    h, npml, core_x, core_y, overlap, wavelengths (and optionally k_coarse, tol, max_iters).
    Raises NosddError (status NOT_CONVERGED) when the forward or the adjoint solve
    stops at max_iters before reaching tol."""
    return _fom_function().apply(eps, J, focal, spec)
