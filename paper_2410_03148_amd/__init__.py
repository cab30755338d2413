"""piezohom: periodic piezoelectric homogenisation on AMD MI355X.

Thin ctypes binding over libpiezohom.so (the C ABI in include/piezohom.h).
Every step of the computation runs in the library's HIP kernels; this
module only marshals arguments.  PyTorch is used, when present, for device
memory and streams (device tensors are passed by pointer).

The library must be built (``python paper_2410_03148_amd/build.py``);
importing the package without it raises ImportError.
"""
from __future__ import annotations

import ctypes as C
import functools
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpiezohom.so")

PHZ_OK = 0
PHZ_NOT_CONVERGED = 1
PHZ_FP64 = 0
PHZ_FP32_IR = 1
PHZ_BF16X3_IR = 2
PHZ_SOLVER_SCP, PHZ_SOLVER_DBP, PHZ_SOLVER_TRICG = 0, 1, 2
PHZ_SMOOTH_ELEMENT, PHZ_SMOOTH_QP = 0, 1
OP_FULL, OP_A, OP_B, OP_SBAR, OP_C, OP_BT = 0, 1, 2, 3, 4, 5


class phz_material(C.Structure):
    _fields_ = [("C", C.c_double * 36), ("e", C.c_double * 18), ("kappa", C.c_double * 9),
                ("void_scale", C.c_double)]


class phz_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("batched", C.c_int), ("restart", C.c_int),
                ("max_iters", C.c_int), ("rtol", C.c_double), ("cheby_degree", C.c_int),
                ("mg_levels", C.c_int), ("smooth_width", C.c_double), ("vcycles_a", C.c_int),
                ("vcycles_s", C.c_int), ("inner_rtol", C.c_double), ("max_refine", C.c_int),
                ("verbose", C.c_int), ("bf16_terms", C.c_int), ("bf16_outer", C.c_int),
                ("elem_tile", C.c_int), ("use_graph", C.c_int), ("fine_kernel", C.c_int),
                ("block_kernel", C.c_int * 4), ("block_tile", C.c_int * 4), ("coarse_kernel", C.c_int),
                ("solver", C.c_int), ("inner", C.c_int), ("inner_eps", C.c_double), ("inner_maxit", C.c_int),
                ("warm_start", C.c_int), ("smoothing", C.c_int),
                ("bf16_terms_precond", C.c_int), ("ir_fallback", C.c_int),
                ("reorth_tol", C.c_double)]


def _set_option(o, k, v):
    if not hasattr(o, k):
        raise TypeError(f"unknown option {k!r}")
    cur = getattr(o, k)
    if isinstance(cur, C.Array):
        if len(v) != len(cur):
            raise ValueError(f"option {k!r} takes {len(cur)} values")
        cur[:] = [int(x) for x in v]
    else:
        setattr(o, k, v)


class phz_stats(C.Structure):
    _fields_ = [("iterations", C.c_int * 9), ("restarts", C.c_int * 9), ("refinements", C.c_int),
                ("true_residual", C.c_double * 9), ("flux_energy_defect", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("mg_levels", C.c_int),
                ("cheb_lambda", C.c_double * 16), ("elem_tile", C.c_int * 4),
                ("fine_kernel", C.c_int * 4), ("coarse_kernel", C.c_int * 16), ("inner_iters", C.c_long * 2),
                ("inner_calls", C.c_long * 2), ("final_precision", C.c_int), ("fallbacks", C.c_int),
                ("reorth_passes", C.c_long)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class phz_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class TorchAllocator:
    """Routes a context's device workspaces through PyTorch's caching allocator
    (phz_allocator callbacks).  Keeps the callbacks alive while the context
    lives; counts calls and bytes outstanding."""

    def __init__(self, device=None):
        import torch
        self._torch = torch
        self.device = torch.cuda.current_device() if device is None else device
        self.allocs = 0
        self.frees = 0
        self.live = {}
        self._alloc = ALLOC_FN(self._do_alloc)
        self._free = FREE_FN(self._do_free)
        self.struct = phz_allocator(self._alloc, self._free, None)

    def _do_alloc(self, nbytes, stream, user):
        try:
            p = self._torch.cuda.caching_allocator_alloc(int(nbytes), device=self.device, stream=stream or 0)
        except Exception:   # out of memory: the library reports PHZ_E_OOM
            return None
        self.allocs += 1
        self.live[p] = int(nbytes)
        return p

    def _do_free(self, ptr, stream, user):
        self.frees += 1
        self.live.pop(ptr, None)
        self._torch.cuda.caching_allocator_delete(ptr)

    @property
    def bytes_live(self):
        return sum(self.live.values())


class phz_foms_t(C.Structure):
    _fields_ = [("d_h", C.c_double), ("g_h", C.c_double), ("B_voigt", C.c_double),
                ("B_reuss", C.c_double), ("k_h", C.c_double)]


EXPORTS = [
    "phz_default_options", "phz_create", "phz_destroy", "phz_last_error", "phz_strerror",
    "phz_set_options", "phz_set_levelset", "phz_set_density", "phz_get_scale", "phz_solve",
    "phz_get_effective", "phz_get_effective_nd", "phz_get_history", "phz_get_stats",
    "phz_get_solution", "phz_set_initial_guess", "phz_get_rhs", "phz_foms", "phz_backward",
    "phz_hj_step", "phz_apply", "phz_precondition", "phz_coarse_apply", "phz_reinit", "phz_levelset_gradient",
    "phz_riesz", "phz_hpm_velocity",
    "phz_kernel_timing", "phz_get_kernel_timing", "phz_orthogonalize", "phz_hj_step_noalloc",
]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2410_03148_amd/build.py`")
    lib = C.CDLL(LIB_PATH)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.c_int
    sig = {
        "phz_default_options": (None, [C.POINTER(phz_options)]),
        "phz_create": (ip, [ip, ip, ip, C.POINTER(phz_material), C.POINTER(phz_options), vp,
                            C.POINTER(phz_allocator), C.POINTER(vp)]),
        "phz_destroy": (None, [vp]),
        "phz_last_error": (C.c_char_p, [vp]),
        "phz_strerror": (C.c_char_p, [ip]),
        "phz_set_options": (ip, [vp, C.POINTER(phz_options)]),
        "phz_set_levelset": (ip, [vp, vp, ip]),
        "phz_set_density": (ip, [vp, vp, ip]),
        "phz_get_scale": (ip, [vp, vp, ip]),
        "phz_solve": (ip, [vp]),
        "phz_get_effective": (ip, [vp, dp, dp, dp]),
        "phz_get_effective_nd": (ip, [vp, dp, dp]),
        "phz_get_history": (ip, [vp, ip, dp, ip, C.POINTER(ip)]),
        "phz_get_stats": (ip, [vp, C.POINTER(phz_stats)]),
        "phz_get_solution": (ip, [vp, vp, ip]),
        "phz_set_initial_guess": (ip, [vp, vp, ip]),
        "phz_get_rhs": (ip, [vp, vp, ip]),
        "phz_foms": (ip, [dp, dp, dp, C.POINTER(phz_foms_t), C.c_char_p, dp, dp, dp]),
        "phz_backward": (ip, [vp, dp, dp, dp, vp, vp, ip]),
        "phz_hj_step": (ip, [vp, vp, C.c_double, vp, ip]),
        "phz_apply": (ip, [vp, ip, ip, ip, vp, vp]),
        "phz_precondition": (ip, [vp, ip, vp, vp]),
        "phz_coarse_apply": (ip, [vp, ip, ip, ip, ip, vp, vp]),
        "phz_reinit": (ip, [vp, ip, C.c_double, ip, vp, ip]),
        "phz_levelset_gradient": (ip, [vp, vp, vp, ip]),
        "phz_riesz": (ip, [vp, ip, C.c_double, vp, vp, C.POINTER(ip)]),
        "phz_hpm_velocity": (ip, [vp, ip, vp, C.POINTER(C.c_void_p), vp, C.c_double, C.c_double, C.c_double,
                                  C.c_double, vp, ip]),
        "phz_kernel_timing": (ip, [vp, ip]),
        "phz_orthogonalize": (ip, [vp, ip, ip, vp, vp, dp, dp, C.POINTER(ip)]),
        "phz_hj_step_noalloc": (ip, [ip, vp, vp, C.c_double, vp, vp]),
        "phz_get_kernel_timing": (ip, [vp, C.c_char_p, ip, C.POINTER(ip)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def _current_device():
    """Index of the current HIP device as torch sees it, or None without torch or a GPU."""
    try:
        import torch
    except ImportError:
        return None
    return torch.cuda.current_device() if torch.cuda.is_available() else None


class PiezoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_lib.phz_strerror(status).decode()} ({status}): {msg}")
        self.status = status


def default_options(**overrides):
    o = phz_options()
    _lib.phz_default_options(C.byref(o))
    for k, v in overrides.items():
        _set_option(o, k, v)
    return o


def make_material(mat):
    """phz_material from an object with C, e, kappa, void_scale (SI)."""
    m = phz_material()
    m.C[:] = [float(v) for v in np.asarray(mat.C, dtype=np.float64).ravel()]
    m.e[:] = [float(v) for v in np.asarray(mat.e, dtype=np.float64).ravel()]
    m.kappa[:] = [float(v) for v in np.asarray(mat.kappa, dtype=np.float64).ravel()]
    m.void_scale = float(mat.void_scale)
    return m


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _is_tensor(buf):
    return hasattr(buf, "data_ptr") and hasattr(buf, "is_cuda")


def _arg(buf, n, device=None, out=False, what="array"):
    """(pointer, on_device, keepalive) for a host array or a device tensor of n float64 values.

    A device tensor passes by pointer, so it must be float64, contiguous, hold exactly n values and
    live on the context's device (index `device`); anything else raises ValueError before the
    library is called.  A host input is converted to a contiguous float64 copy; a host output
    (out=True) must already be a contiguous float64 array (or CPU tensor) of n values, because the
    library writes into its memory."""
    if _is_tensor(buf):
        if buf.is_cuda:
            import torch
            if buf.dtype != torch.float64:
                raise ValueError(f"{what}: device tensor must be float64, got {buf.dtype}")
            if not buf.is_contiguous():
                raise ValueError(f"{what}: device tensor must be contiguous")
            if buf.numel() != n:
                raise ValueError(f"{what}: device tensor must hold {n} values, got {buf.numel()}")
            if device is not None and buf.device.index != device:
                raise ValueError(f"{what}: tensor on cuda:{buf.device.index}, context on cuda:{device}")
            return C.c_void_p(buf.data_ptr()), 1, buf
        if out:
            import torch
            if buf.dtype != torch.float64 or not buf.is_contiguous() or buf.numel() != n:
                raise ValueError(f"{what}: output tensor must be contiguous float64 with {n} values")
            a = buf.numpy()
            return C.c_void_p(a.ctypes.data), 0, a
        buf = buf.detach().numpy()
    if out:
        if not isinstance(buf, np.ndarray) or buf.dtype != np.float64 or not buf.flags.c_contiguous \
                or buf.size != n or not buf.flags.writeable:
            raise ValueError(f"{what}: output array must be a writable contiguous float64 array of {n} values")
        return C.c_void_p(buf.ctypes.data), 0, buf
    a = np.ascontiguousarray(buf, dtype=np.float64).ravel()
    if a.size != n:
        raise ValueError(f"{what}: expected {n} values, got {a.size}")
    return C.c_void_p(a.ctypes.data), 0, a


def foms(CH, eH, kH, grad_of=None):
    """Figures of merit (d_h, g_h, B_voigt, B_reuss, k_h) and optional gradients."""
    CH = np.ascontiguousarray(CH, dtype=np.float64).ravel()
    eH = np.ascontiguousarray(eH, dtype=np.float64).ravel()
    kH = np.ascontiguousarray(kH, dtype=np.float64).ravel()
    out = phz_foms_t()
    gC, ge, gk = np.zeros(36), np.zeros(18), np.zeros(9)
    st = _lib.phz_foms(_dptr(CH), _dptr(eH), _dptr(kH), C.byref(out),
                       grad_of.encode() if grad_of else None, _dptr(gC), _dptr(ge), _dptr(gk))
    if st != PHZ_OK:
        raise PiezoError(st, "phz_foms")
    f = {k: getattr(out, k) for k in ("d_h", "g_h", "B_voigt", "B_reuss", "k_h")}
    if grad_of:
        return f, (gC.reshape(6, 6), ge.reshape(3, 6), gk.reshape(3, 3))
    return f


class Context:
    """One periodic N^3 cell on the GPU (wraps phz_ctx)."""

    def __init__(self, n, material, stream=None, allocator=None, **opts):
        """allocator: None (the library's hipMalloc), "torch" (PyTorch's caching
        allocator, through TorchAllocator) or a TorchAllocator."""
        self.n = n
        self.nn = n ** 3
        self._mat = make_material(material)
        self._opt = default_options(**opts)
        self.device = _current_device()
        self._state = 0    # advances whenever the geometry or the solution may change
        if allocator == "torch":
            allocator = TorchAllocator(self.device)
        self.allocator = allocator
        h = C.c_void_p()
        st = _lib.phz_create(n, n, n, C.byref(self._mat), C.byref(self._opt),
                             C.c_void_p(stream) if stream else None,
                             C.byref(allocator.struct) if allocator is not None else None, C.byref(h))
        if st != PHZ_OK:
            raise PiezoError(st, "phz_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.phz_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st, what, allow_nc=False):
        if st == PHZ_OK or (allow_nc and st == PHZ_NOT_CONVERGED):
            return st
        raise PiezoError(st, f"{what}: {_lib.phz_last_error(self._h).decode()}")

    def set_options(self, **opts):
        for k, v in opts.items():
            _set_option(self._opt, k, v)
        self._state += 1
        self._check(_lib.phz_set_options(self._h, C.byref(self._opt)), "phz_set_options")

    def set_levelset(self, phi):
        p, dev, keep = _arg(phi, self.nn, self.device, what="set_levelset")
        self._state += 1
        self._check(_lib.phz_set_levelset(self._h, p, dev), "phz_set_levelset")

    def set_density(self, rho):
        p, dev, keep = _arg(rho, self.nn, self.device, what="set_density")
        self._state += 1
        self._check(_lib.phz_set_density(self._h, p, dev), "phz_set_density")

    def scale(self, out=None):
        """Element scales s_e (host array, or into `out`: a host array or a device tensor)."""
        if out is None:
            out = np.zeros(self.nn)
        p, dev, _ = _arg(out, self.nn, self.device, out=True, what="scale(out=)")
        self._check(_lib.phz_get_scale(self._h, p, dev), "phz_get_scale")
        return out

    def solve(self):
        """Solve the nine cell problems; returns PHZ_OK or PHZ_NOT_CONVERGED."""
        self._state += 1
        return self._check(_lib.phz_solve(self._h), "phz_solve", allow_nc=True)

    def effective(self):
        Cm, e, k = np.zeros(36), np.zeros(18), np.zeros(9)
        self._check(_lib.phz_get_effective(self._h, _dptr(Cm), _dptr(e), _dptr(k)), "phz_get_effective")
        return Cm.reshape(6, 6), e.reshape(3, 6), k.reshape(3, 3)

    def effective_nd(self):
        a, b = np.zeros(81), np.zeros(81)
        self._check(_lib.phz_get_effective_nd(self._h, _dptr(a), _dptr(b)), "phz_get_effective_nd")
        return a.reshape(9, 9), b.reshape(9, 9)

    def stats(self):
        s = phz_stats()
        self._check(_lib.phz_get_stats(self._h, C.byref(s)), "phz_get_stats")
        return {
            "iterations": list(s.iterations), "restarts": list(s.restarts),
            "refinements": s.refinements, "true_residual": list(s.true_residual),
            "flux_energy_defect": s.flux_energy_defect, "setup_ms": s.setup_ms,
            "solve_ms": s.solve_ms, "mg_levels": s.mg_levels,
            "cheb_lambda": list(s.cheb_lambda), "elem_tile": list(s.elem_tile),
            "fine_kernel": list(s.fine_kernel), "coarse_kernel": list(s.coarse_kernel),
            "inner_iters": list(s.inner_iters), "inner_calls": list(s.inner_calls),
            "final_precision": s.final_precision, "fallbacks": s.fallbacks, "reorth_passes": s.reorth_passes,
        }

    def history(self, load):
        n = C.c_int()
        self._check(_lib.phz_get_history(self._h, load, None, 0, C.byref(n)), "phz_get_history")
        buf = np.zeros(max(n.value, 1))
        self._check(_lib.phz_get_history(self._h, load, _dptr(buf), n.value, C.byref(n)), "phz_get_history")
        return buf[: n.value]

    def solution(self, out=None):
        """X as [N^3, 4, 9] (host numpy, or into a device tensor `out`)."""
        if out is not None:
            p, dev, keep = _arg(out, self.nn * 36, self.device, out=True, what="solution(out=)")
            self._check(_lib.phz_get_solution(self._h, p, dev), "phz_get_solution")
            return out
        X = np.zeros(self.nn * 36)
        self._check(_lib.phz_get_solution(self._h, C.c_void_p(X.ctypes.data), 0), "phz_get_solution")
        return X.reshape(self.nn, 4, 9)

    def set_initial_guess(self, X):
        if X is None:
            self._check(_lib.phz_set_initial_guess(self._h, None, 0), "phz_set_initial_guess")
            return
        p, dev, keep = _arg(X, self.nn * 36, self.device, what="set_initial_guess")
        self._check(_lib.phz_set_initial_guess(self._h, p, dev), "phz_set_initial_guess")

    def rhs(self):
        b = np.zeros(self.nn * 36)
        self._check(_lib.phz_get_rhs(self._h, C.c_void_p(b.ctypes.data), 0), "phz_get_rhs")
        return b.reshape(self.nn, 4, 9)

    def backward(self, gC=None, ge=None, gk=None, want_phi=False, out_rho=None, out_phi=None):
        """dJ/drho (and dJ/dphi) for upstream gradients w.r.t. (C^H, e^H, kappa^H)."""
        z = lambda a, n: np.ascontiguousarray(np.zeros(n) if a is None else a, dtype=np.float64).ravel()
        gC, ge, gk = z(gC, 36), z(ge, 18), z(gk, 9)
        if out_rho is not None:
            prho, dev, _ = _arg(out_rho, self.nn, self.device, out=True, what="backward(out_rho=)")
            pphi = None
            if out_phi is not None:
                pphi, dphi, _ = _arg(out_phi, self.nn, self.device, out=True, what="backward(out_phi=)")
                if dphi != dev:
                    raise ValueError("backward: out_rho and out_phi must both be on the host or both on the device")
            self._check(_lib.phz_backward(self._h, _dptr(gC), _dptr(ge), _dptr(gk), prho, pphi, dev), "phz_backward")
            return out_rho, out_phi
        grho = np.zeros(self.nn)
        gphi = np.zeros(self.nn) if want_phi else None
        self._check(_lib.phz_backward(self._h, _dptr(gC), _dptr(ge), _dptr(gk), C.c_void_p(grho.ctypes.data),
                                      C.c_void_p(gphi.ctypes.data) if want_phi else None, 0), "phz_backward")
        return (grho, gphi) if want_phi else grho

    def hj_step(self, velocity=None, cfl=0.5, return_phi=True, out=None):
        """One HJ step; velocity None uses the last backward's dJ/drho.  A device velocity
        tensor keeps the step on the device; `out` (a device tensor) receives the new level set
        there instead of a returned host copy."""
        on_dev = (velocity is not None and _is_tensor(velocity) and velocity.is_cuda) or \
            (out is not None and _is_tensor(out) and out.is_cuda)
        if on_dev:
            pv = None
            if velocity is not None:
                pv, dv, keep_v = _arg(velocity, self.nn, self.device, what="hj_step(velocity)")
                if not dv:
                    raise ValueError("hj_step: with a device output the velocity must be on the device too")
            po = None
            if out is not None:
                po, do, _ = _arg(out, self.nn, self.device, out=True, what="hj_step(out=)")
                if not do:
                    raise ValueError("hj_step: out must be a device tensor when the velocity is one")
            st = _lib.phz_hj_step(self._h, pv, cfl, po, 1)
            self._state += 1
            self._check(st, "phz_hj_step")
            return out
        out = np.zeros(self.nn) if return_phi else None
        optr = C.c_void_p(out.ctypes.data) if return_phi else None
        if velocity is None:
            st = _lib.phz_hj_step(self._h, None, cfl, optr, 0)
        else:
            v = np.ascontiguousarray(velocity, dtype=np.float64).ravel()
            if v.size != self.nn:
                raise ValueError(f"hj_step: velocity must hold {self.nn} values")
            st = _lib.phz_hj_step(self._h, C.c_void_p(v.ctypes.data), cfl, optr, 0)
        self._state += 1
        self._check(st, "phz_hj_step")
        return out

    def reinit(self, steps=20, cfl=0.5, subcell=False, return_phi=True):
        """Reinitialise the level set towards a signed distance (phz_reinit; subcell: Russo-Smereka fix)."""
        out = np.zeros(self.nn) if return_phi else None
        self._state += 1
        self._check(_lib.phz_reinit(self._h, steps, cfl, 1 if subcell else 0,
                                    C.c_void_p(out.ctypes.data) if return_phi else None, 0), "phz_reinit")
        return out

    def levelset_gradient(self, grad_rho, out=None):
        """dJ/dphi from an element gradient dJ/drho (phz_levelset_gradient); with a device tensor
        grad_rho, into the device tensor `out`."""
        if _is_tensor(grad_rho) and grad_rho.is_cuda:
            pg, _, _ = _arg(grad_rho, self.nn, self.device, what="levelset_gradient(grad_rho)")
            if out is None:
                raise ValueError("levelset_gradient: a device grad_rho needs a device `out`")
            po, do, _ = _arg(out, self.nn, self.device, out=True, what="levelset_gradient(out=)")
            if not do:
                raise ValueError("levelset_gradient: `out` must be a device tensor")
            self._check(_lib.phz_levelset_gradient(self._h, pg, po, 1), "phz_levelset_gradient")
            return out
        g = np.ascontiguousarray(grad_rho, dtype=np.float64).ravel()
        if g.size != self.nn:
            raise ValueError(f"levelset_gradient: grad_rho must hold {self.nn} values")
        out = np.zeros(self.nn)
        self._check(_lib.phz_levelset_gradient(self._h, _dptr(g), C.c_void_p(out.ctypes.data), 0),
                    "phz_levelset_gradient")
        return out

    def riesz(self, ncol, alpha, j_ptr, g_ptr):
        """g = (alpha^2 K + M)^-1 j on ncol device node columns; returns the iterations."""
        it = C.c_int()
        self._check(_lib.phz_riesz(self._h, ncol, alpha, C.c_void_p(j_ptr), C.c_void_p(g_ptr), C.byref(it)),
                    "phz_riesz")
        return it.value

    def hpm_velocity(self, j_obj, j_cons=(), viol=(), alpha=0.0, cfl=0.5, gamma=0.5, obj_weight=1.0, out=None):
        """Velocity of one constrained step (phz_hpm_velocity): host arrays, or device tensors (j_obj,
        every j_cons and `out`; the violations stay on the host)."""
        if _is_tensor(j_obj) and j_obj.is_cuda:
            pj, _, _ = _arg(j_obj, self.nn, self.device, what="hpm_velocity(j_obj)")
            cons = [_arg(j, self.nn, self.device, what="hpm_velocity(j_cons)") for j in j_cons]
            if any(not d for _, d, _ in cons):
                raise ValueError("hpm_velocity: with a device j_obj every j_cons must be a device tensor")
            vi = np.ascontiguousarray(viol, dtype=np.float64).ravel()
            if vi.size != len(cons):
                raise ValueError("hpm_velocity: one violation per constraint")
            if out is None:
                raise ValueError("hpm_velocity: device inputs need a device `out`")
            po, do, _ = _arg(out, self.nn, self.device, out=True, what="hpm_velocity(out=)")
            if not do:
                raise ValueError("hpm_velocity: `out` must be a device tensor")
            ptrs = (C.c_void_p * max(len(cons), 1))(*[p.value for p, _, _ in cons])
            self._check(_lib.phz_hpm_velocity(self._h, len(cons), pj, ptrs,
                                              _dptr(vi) if len(cons) else None, alpha, cfl, gamma, obj_weight, po, 1),
                        "phz_hpm_velocity")
            return out
        jo = np.ascontiguousarray(j_obj, dtype=np.float64).ravel()
        jc = [np.ascontiguousarray(j, dtype=np.float64).ravel() for j in j_cons]
        vi = np.ascontiguousarray(viol, dtype=np.float64).ravel()
        if jo.size != self.nn or any(j.size != self.nn for j in jc) or vi.size != len(jc):
            raise ValueError(f"hpm_velocity: node columns of {self.nn} values and one violation per constraint")
        ptrs = (C.c_void_p * max(len(jc), 1))(*[j.ctypes.data for j in jc])
        out = np.zeros(self.nn)
        self._check(_lib.phz_hpm_velocity(self._h, len(jc), _dptr(jo), ptrs, _dptr(vi) if len(jc) else None,
                                          alpha, cfl, gamma, obj_weight, C.c_void_p(out.ctypes.data), 0),
                    "phz_hpm_velocity")
        return out

    def kernel_timing(self, enable=True, fine_only=False):
        """Enable (or disable) per-kernel HIP-event timing; clears the totals.
        fine_only: bracket the fine-level operator launches only."""
        self._check(_lib.phz_kernel_timing(self._h, (2 if fine_only else 1) if enable else 0), "phz_kernel_timing")

    def kernel_times(self):
        """{name: (launches, total_ms)} recorded since timing was enabled."""
        n = C.c_int()
        self._check(_lib.phz_get_kernel_timing(self._h, None, 0, C.byref(n)), "phz_get_kernel_timing")
        buf = C.create_string_buffer(n.value + 1)
        self._check(_lib.phz_get_kernel_timing(self._h, buf, n.value + 1, C.byref(n)), "phz_get_kernel_timing")
        out = {}
        for line in buf.value.decode().splitlines():
            name, cnt, ms = line.split()
            out[name] = (int(cnt), float(ms))
        return out

    # ---- low-level device entry points (pointers to device memory) ----
    def apply(self, op, nrhs, precision, x_ptr, y_ptr):
        self._check(_lib.phz_apply(self._h, op, nrhs, precision, C.c_void_p(x_ptr), C.c_void_p(y_ptr)),
                    "phz_apply")

    def precondition(self, nrhs, r_ptr, z_ptr):
        self._check(_lib.phz_precondition(self._h, nrhs, C.c_void_p(r_ptr), C.c_void_p(z_ptr)),
                    "phz_precondition")

    def orthogonalize(self, precision, nvec, V_ptr, w_ptr):
        """One Arnoldi orthogonalisation of w (device) against nvec basis vectors V (device);
        returns (h [nvec, 9], |w|^2 [9], second pass taken [9])."""
        h = np.zeros(nvec * 9)
        n2 = np.zeros(9)
        sp = (C.c_int * 9)()
        self._check(_lib.phz_orthogonalize(self._h, precision, nvec, C.c_void_p(V_ptr), C.c_void_p(w_ptr), _dptr(h),
                                           _dptr(n2), sp), "phz_orthogonalize")
        return h.reshape(nvec, 9), n2, np.array(list(sp))

    def coarse_apply(self, level, op, nrhs, x_ptr, y_ptr, precision=PHZ_FP64):
        self._check(_lib.phz_coarse_apply(self._h, level, op, nrhs, precision, C.c_void_p(x_ptr),
                                          C.c_void_p(y_ptr)), "phz_coarse_apply")


def hj_step_noalloc(n, phi, grad_rho, cfl, phi_out, stream=None):
    """phz_hj_step_noalloc: one HJ step of the device level set phi driven by the
    device element gradient grad_rho, into the device tensor phi_out, on `stream`
    (a HIP stream handle; None the default stream).  Allocates nothing."""
    nn = n ** 3
    pp, dp_, _ = _arg(phi, nn, what="hj_step_noalloc(phi)")
    pg, dg, _ = _arg(grad_rho, nn, what="hj_step_noalloc(grad_rho)")
    po, do, _ = _arg(phi_out, nn, out=True, what="hj_step_noalloc(phi_out)")
    if not (dp_ and dg and do):
        raise ValueError("hj_step_noalloc: phi, grad_rho and phi_out must be device tensors")
    st = _lib.phz_hj_step_noalloc(n, pp, pg, float(cfl), po, C.c_void_p(stream) if stream else None)
    if st != PHZ_OK:
        raise PiezoError(st, _lib.phz_last_error(None).decode())


def homogenise(n, material, phi=None, rho=None, **opts):
    """Solve one cell and return a dict of SI tensors, FOMs and solver stats."""
    with Context(n, material, **opts) as ctx:
        if phi is not None:
            ctx.set_levelset(phi)
        else:
            ctx.set_density(rho)
        status = ctx.solve()
        Cm, e, k = ctx.effective()
        return {"C": Cm, "e": e, "kappa": k, "foms": foms(Cm, e, k), "stats": ctx.stats(),
                "status": status}


@functools.lru_cache(maxsize=None)
def _autograd():
    import torch

    class Homogenise(torch.autograd.Function):
        """(C^H, e^H, kappa^H) = F(rho) with a hand-written backward.

        forward: rho (float64 tensor [N^3] on the context's device, or on
        the host) -> three float64 CPU tensors (SI); it raises if the solve
        does not converge.  backward: phz_backward turns the upstream
        gradients into dJ/drho on rho's device.  The backward uses the
        solution the context holds, so it raises if the context has been
        given a new geometry, options or solve since this forward.
        """

        @staticmethod
        def forward(ctx_, rho, context):
            context.set_density(rho.detach())
            status = context.solve()
            if status != PHZ_OK:
                raise PiezoError(status, "Homogenise: the cell solve did not converge")
            Cm, e, k = context.effective()
            ctx_.context = context
            ctx_.state = context._state
            ctx_.device = rho.device
            return (torch.from_numpy(Cm.copy()), torch.from_numpy(e.copy()), torch.from_numpy(k.copy()))

        @staticmethod
        def backward(ctx_, gC, ge, gk):
            context = ctx_.context
            if context._state != ctx_.state:
                raise RuntimeError("Homogenise.backward: the context changed since this forward "
                                   "(a new geometry, options or solve); run the forward again")
            cvt = lambda g: None if g is None else g.detach().cpu().double().numpy()
            if ctx_.device.type == "cuda":
                out = torch.empty(context.nn, dtype=torch.float64, device=ctx_.device)
                context.backward(cvt(gC), cvt(ge), cvt(gk), out_rho=out)
                return out, None
            g = context.backward(cvt(gC), cvt(ge), cvt(gk))
            return torch.from_numpy(g), None

    return Homogenise


def __getattr__(name):
    if name == "Homogenise":
        return _autograd()
    raise AttributeError(name)
