"""ctypes binding of libfc2d.so (argument marshalling only; every step runs in
the library's HIP kernels).  Names follow include/fc2d.h.

Device buffers are torch tensors (float64, contiguous, on the current HIP
device); streams default to torch's current stream.  The library must have
been built (``python -m paper_2010_03901_amd.build``); nothing here computes
a fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfc2d.so")

FC2D_OK = 0
FC2D_E_ARG, FC2D_E_TABLE, FC2D_E_GEOMETRY, FC2D_E_NEWTON, FC2D_E_HIP, FC2D_E_NOMEM = -1, -2, -3, -4, -5, -6
FC2D_CURVE_POLAR, FC2D_CURVE_CARTESIAN = 1, 2
FC2D_FORWARD, FC2D_INVERSE = -1, 1
FC2D_LAPLACE_INV, FC2D_DX, FC2D_DY = 1, 2, 3
FC2D_TUNE_COL_TILE, FC2D_TUNE_STRIP_FIELDS, FC2D_TUNE_COL_ELEMS, FC2D_TUNE_STRIP_WINDOW, FC2D_TUNE_FF_SHAPE = 1, 2, 3, 4, 5
FC2D_BATCH_AUTOTUNE, FC2D_BATCH_FUSED_FF, FC2D_BATCH_TRANSPOSED = 1, 2, 4
FC2D_SEED_PROXIMITY, FC2D_SEED_POLAR, FC2D_SEED_MLP = 0, 1, 2
FC2D_MLP_NIN, FC2D_MLP_HIDDEN, FC2D_MLP_NW = 8, 64, 9026

FAR, IN, STRIP = 0, 1, 2


class Fc2dError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (_lib().fc2d_strerror(status).decode(), status, msg))
        self.status = status


class fc2d_curve(C.Structure):
    _fields_ = [("kind", C.c_int), ("nmodes", C.c_int), ("a", C.POINTER(C.c_double)), ("b", C.POINTER(C.c_double))]


class fc2d_grid(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("h", C.c_double), ("nx", C.c_int), ("ny", C.c_int)]


class fc2d_opts(C.Structure):
    _fields_ = [("B", C.c_int), ("k1", C.c_double), ("M", C.c_int), ("n_r", C.c_int), ("Z", C.c_int),
                ("n_os", C.c_int), ("mf", C.c_int), ("newton_maxit", C.c_int), ("seed", C.c_int),
                ("mlp_tol", C.c_double), ("mlp_weights", C.POINTER(C.c_float)), ("interior_only", C.c_int)]


class fc2d_plan_info(C.Structure):
    _fields_ = [("d", C.c_int), ("C", C.c_int), ("M", C.c_int), ("n_r", C.c_int), ("Cr", C.c_int), ("B", C.c_int),
                ("k1", C.c_double), ("k2", C.c_double), ("n_bdry", C.c_int64), ("n_strip", C.c_int64),
                ("n_in", C.c_int64), ("n_far", C.c_int64), ("newton_max_iters", C.c_int), ("seed", C.c_int),
                ("n_solved", C.c_int64), ("n_fallback", C.c_int64), ("newton_iters", C.c_int64),
                ("t_ms", C.c_double * 5)]

# fc2d_plan_info.t_ms phases
PLAN_PHASES = ("geometry", "classify", "lists", "matching", "layout")


class fc2d_ff_info(C.Structure):
    _fields_ = [("c", C.c_double), ("dT", C.c_double), ("dt", C.c_double), ("K", C.c_int), ("n_c", C.c_int),
                ("M_b", C.c_int), ("n_cross", C.c_int64), ("n_stepped", C.c_int64), ("n_bnd", C.c_int64),
                ("n_segments", C.c_int), ("max_segment", C.c_int)]


_LIB = None
_P = C.c_void_p


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libfc2d.so is not built; run `python -m paper_2010_03901_amd.build`")
        lib = C.CDLL(LIB_PATH)
        sig = {
            "fc2d_opts_default": (None, [C.POINTER(fc2d_grid), C.POINTER(fc2d_opts)]),
            "fc2d_plan_create": (C.c_int, [C.POINTER(fc2d_curve), C.POINTER(fc2d_grid), C.c_int, C.c_int,
                                           C.POINTER(fc2d_opts), _P, C.POINTER(_P)]),
            "fc2d_plan_destroy": (C.c_int, [_P]),
            "fc2d_plan_get_info": (C.c_int, [_P, C.POINTER(fc2d_plan_info)]),
            "fc2d_boundary_points": (C.c_int, [_P, C.POINTER(C.c_int64), _P]),
            "fc2d_plan_classes": (C.c_int, [_P, _P]),
            "fc2d_plan_strip": (C.c_int, [_P, _P, _P, _P, _P]),
            "fc2d_matching": (C.c_int, [_P, _P, _P, _P, C.c_int, _P]),
            "fc2d_blend": (C.c_int, [_P, _P, _P, _P, C.c_int, _P]),
            "fc2d_extend": (C.c_int, [_P, _P, _P, _P, C.c_int, _P]),
            "fc2d_extend_fft": (C.c_int, [_P, _P, _P, _P, _P, C.c_int, _P]),
            "fc2d_extend_fft_noalloc": (C.c_int, [_P, _P, _P, _P, _P, C.c_int, _P]),
            "fc2d_extend_fft_ld": (C.c_int, [_P, _P, _P, _P, _P, C.c_int, C.c_int, _P]),
            "fc2d_fft_ld": (C.c_int, [C.POINTER(fc2d_grid), _P, _P, C.c_int, C.c_int, C.c_int, _P]),
            "fc2d_fft": (C.c_int, [C.POINTER(fc2d_grid), _P, _P, C.c_int, C.c_int, _P]),
            "fc2d_spectral_apply": (C.c_int, [C.POINTER(fc2d_grid), C.c_int, _P, _P, C.c_int, _P]),
            "fc2d_poisson_nodes": (C.c_int, [_P, C.c_int, _P]),
            "fc2d_poisson_solve": (C.c_int, [_P, _P, _P, _P, C.c_int, _P, C.c_int, _P, C.POINTER(C.c_int)]),
            "ff_propagate": (C.c_int, [C.POINTER(fc2d_grid), C.c_double, C.c_double, _P, _P, _P, _P, C.c_int, _P]),
            "fc2d_boundary_values": (C.c_int, [_P, _P, _P, C.c_int, _P]),
            "fc2d_batch_create": (C.c_int, [C.POINTER(_P), C.POINTER(C.c_int), C.c_int, C.c_uint, _P, C.POINTER(_P)]),
            "fc2d_batch_state": (C.c_int, [_P, C.c_int, C.POINTER(_P), C.POINTER(_P)]),
            "fc2d_batch_info": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
            "fc2d_batch_run_ff": (C.c_int, [_P, C.c_double, C.c_double, C.c_int, C.c_int, _P]),
            "fc2d_batch_destroy": (C.c_int, [_P]),
            "fc2d_tune_set": (C.c_int, [C.c_int, C.c_int, C.c_int]),
            "fc2d_tune_get": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int)]),
            "fc2d_trace_begin": (C.c_int, [_P]),
            "fc2d_trace_end": (C.c_int, [C.POINTER(C.c_int), C.POINTER(C.c_char_p), C.POINTER(C.c_float), C.c_int]),
            "fc2d_mlp_make_data": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P, C.c_int64, C.c_double, _P, _P, _P,
                                             _P, _P]),
            "fc2d_mlp_forward": (C.c_int, [_P, _P, C.c_int64, _P, _P]),
            "fc2d_mlp_loss_grad": (C.c_int, [_P, _P, _P, C.c_int64, _P, _P, _P]),
            "fc2d_mlp_train": (C.c_int, [_P, _P, _P, _P, _P, C.c_int64, C.c_int, C.c_int, C.c_int64, C.c_float,
                                         C.c_float, C.c_int64, _P, _P]),
            "fc2d_ff_create": (C.c_int, [_P, C.c_double, C.c_int, C.c_int, _P, C.POINTER(_P)]),
            "fc2d_ff_destroy": (C.c_int, [_P]),
            "fc2d_ff_get_info": (C.c_int, [_P, C.POINTER(fc2d_ff_info)]),
            "fc2d_ff_crossings": (C.c_int, [_P, C.POINTER(C.c_int64), _P]),
            "fc2d_ff_regions": (C.c_int, [_P, _P]),
            "fc2d_ff_advance": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, C.c_int, _P]),
            "fc2d_strerror": (C.c_char_p, [C.c_int]),
            "fc2d_last_error": (C.c_char_p, []),
            "fc2d_version": (C.c_int, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def _check(status):
    if status != FC2D_OK:
        raise Fc2dError(status, _lib().fc2d_last_error().decode())


def _stream(stream):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t, name, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise TypeError("%s must be %s" % (name, dtype))
    return C.c_void_p(t.data_ptr())


def _bptr(plan, f_bdry):
    """Boundary samples: a device tensor, or None for a plan built from interior data only."""
    if f_bdry is None:
        if not plan.interior_only:
            raise TypeError("f_bdry is required unless the plan was built with interior_only=True")
        return None
    return _dptr(f_bdry, "f_bdry", __import__("torch").float64)


def make_grid(x0, y0, h, nx, ny):
    return fc2d_grid(float(x0), float(y0), float(h), int(nx), int(ny))


def make_curve(kind, coef):
    """kind 'polar' with coef [c0, a1, b1, ...] or 'cartesian' with ([x...], [y...])."""
    if kind == "polar":
        a = np.ascontiguousarray(coef, dtype=np.float64)
        b = None
        k = FC2D_CURVE_POLAR
    else:
        xa, ya = coef
        n = max(len(xa), len(ya))
        a = np.zeros(n)
        b = np.zeros(n)
        a[: len(xa)] = xa
        b[: len(ya)] = ya
        k = FC2D_CURVE_CARTESIAN
    if a.size % 2 == 0:
        a = np.concatenate([a, [0.0]])
        if b is not None:
            b = np.concatenate([b, [0.0]])
    nm = (a.size - 1) // 2
    cv = fc2d_curve(k, nm, a.ctypes.data_as(C.POINTER(C.c_double)),
                    b.ctypes.data_as(C.POINTER(C.c_double)) if b is not None else None)
    cv._keep = (a, b)
    return cv


class Plan:
    """Owning wrapper of fc2d_plan*."""

    def __init__(self, curve, grid, d=5, C_=27, B=None, k1=None, M=None, n_r=None, Z=None, n_os=None, mf=None,
                 newton_maxit=None, seed=None, mlp_weights=None, mlp_tol=None, interior_only=False, stream=None):
        lib = _lib()
        self.grid = grid
        self.interior_only = bool(interior_only)
        opts = fc2d_opts()
        lib.fc2d_opts_default(C.byref(grid), C.byref(opts))
        for name, v in (("B", B), ("k1", k1), ("M", M), ("n_r", n_r), ("Z", Z), ("n_os", n_os), ("mf", mf),
                        ("newton_maxit", newton_maxit), ("seed", seed), ("mlp_tol", mlp_tol)):
            if v is not None:
                setattr(opts, name, v)
        opts.interior_only = 1 if interior_only else 0
        if mlp_weights is not None:
            wts = np.ascontiguousarray(mlp_weights, dtype=np.float32)
            if wts.size != FC2D_MLP_NW:
                raise ValueError("mlp_weights must hold %d floats" % FC2D_MLP_NW)
            opts.mlp_weights = wts.ctypes.data_as(C.POINTER(C.c_float))
        h = C.c_void_p()
        _check(lib.fc2d_plan_create(C.byref(curve), C.byref(grid), int(d), int(C_), C.byref(opts),
                                    _stream(stream), C.byref(h)))
        self._h = h
        info = fc2d_plan_info()
        _check(lib.fc2d_plan_get_info(h, C.byref(info)))
        self.info = info

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib().fc2d_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fc2d_plan_create(curve, grid, d=5, C_=27, **kw):
    return Plan(curve, grid, d, C_, **kw)


def fc2d_plan_destroy(plan):
    plan.close()


def fc2d_boundary_points(plan):
    n = C.c_int64()
    _check(_lib().fc2d_boundary_points(plan.handle, C.byref(n), None))
    xy = np.zeros((n.value, 2))
    _check(_lib().fc2d_boundary_points(plan.handle, C.byref(n), C.c_void_p(xy.ctypes.data)))
    return xy


def fc2d_plan_classes(plan):
    g = plan.grid
    out = np.zeros((g.nx, g.ny), dtype=np.int8)
    _check(_lib().fc2d_plan_classes(plan.handle, C.c_void_p(out.ctypes.data)))
    return out


def fc2d_plan_strip(plan):
    S = plan.info.n_strip
    idx = np.zeros(S, dtype=np.int64)
    th = np.zeros(S)
    eta = np.zeros(S)
    seed = np.zeros(S, dtype=np.int32)
    _check(_lib().fc2d_plan_strip(plan.handle, C.c_void_p(idx.ctypes.data), C.c_void_p(th.ctypes.data),
                                  C.c_void_p(eta.ctypes.data), C.c_void_p(seed.ctypes.data)))
    return idx, th, eta, seed


def _nf(f_grid, grid):
    n = f_grid.numel() // (grid.nx * grid.ny)
    if n * grid.nx * grid.ny != f_grid.numel():
        raise ValueError("f_grid size is not a multiple of nx*ny")
    return n


def _check_bdry(plan, f_bdry, nf):
    import torch
    if f_bdry is not None and (f_bdry.dtype != torch.float64 or f_bdry.numel() != nf * plan.info.n_bdry):
        raise ValueError("f_bdry must be float64 [nf][n_bdry] with n_bdry = %d" % plan.info.n_bdry)


def _check_out(t, name, numel, dtype):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.numel() != numel:
        raise ValueError("%s must be %s with %d elements" % (name, dtype, numel))


def fc2d_matching(plan, f_grid, f_bdry, fD, stream=None):
    import torch
    nf = _nf(f_grid, plan.grid)
    _check_bdry(plan, f_bdry, nf)
    _check_out(fD, "fD", nf * plan.info.B * plan.info.d, torch.float64)
    _check(_lib().fc2d_matching(plan.handle, _dptr(f_grid, "f_grid", torch.float64), _bptr(plan, f_bdry),
                                _dptr(fD, "fD", torch.float64), nf, _stream(stream)))


def fc2d_blend(plan, f_grid, f_bdry, F, stream=None):
    import torch
    nf = _nf(f_grid, plan.grid)
    _check_bdry(plan, f_bdry, nf)
    _check_out(F, "F", nf * (plan.info.Cr + 1) * plan.info.B, torch.float64)
    _check(_lib().fc2d_blend(plan.handle, _dptr(f_grid, "f_grid", torch.float64), _bptr(plan, f_bdry),
                             _dptr(F, "F", torch.float64), nf, _stream(stream)))


def fc2d_extend(plan, f_grid, f_bdry, out, stream=None):
    import torch
    nf = _nf(f_grid, plan.grid)
    _check_bdry(plan, f_bdry, nf)
    _check_out(out, "out", f_grid.numel(), torch.float64)
    _check(_lib().fc2d_extend(plan.handle, _dptr(f_grid, "f_grid", torch.float64), _bptr(plan, f_bdry),
                              _dptr(out, "out", torch.float64), nf, _stream(stream)))


def _extend_fft_args(plan, f_grid, f_bdry, work, spec):
    import torch
    nf = _nf(f_grid, plan.grid)
    g = plan.grid
    _check_bdry(plan, f_bdry, nf)
    _check_out(work, "work", f_grid.numel(), torch.float64)
    _check_out(spec, "spec", nf * g.nx * (g.ny // 2 + 1), torch.complex128)
    return (plan.handle, _dptr(f_grid, "f_grid", torch.float64), _bptr(plan, f_bdry),
            _dptr(work, "work", torch.float64), _dptr(spec, "spec"), nf)


def fc2d_extend_fft(plan, f_grid, f_bdry, work, spec, stream=None):
    _check(_lib().fc2d_extend_fft(*_extend_fft_args(plan, f_grid, f_bdry, work, spec), _stream(stream)))


def fc2d_extend_fft_ld(plan, f_grid, f_bdry, work, spec, stream=None):
    """fc2d_extend_fft into spec [nf][nx][ld] complex128 (rows ld >= ny/2+1 apart)."""
    import torch
    nf = _nf(f_grid, plan.grid)
    g = plan.grid
    _check_bdry(plan, f_bdry, nf)
    _check_out(work, "work", f_grid.numel(), torch.float64)
    if spec.dtype != torch.complex128 or spec.dim() != 3 or tuple(spec.shape[:2]) != (nf, g.nx) or \
            spec.shape[2] < g.ny // 2 + 1:
        raise ValueError("spec must be complex128 [nf][nx][ld] with ld >= ny/2+1")
    _check(_lib().fc2d_extend_fft_ld(plan.handle, _dptr(f_grid, "f_grid", torch.float64), _bptr(plan, f_bdry),
                                     _dptr(work, "work", torch.float64), _dptr(spec, "spec"), int(spec.shape[2]), nf,
                                     _stream(stream)))


def fc2d_fft_ld(grid, inp, out, direction, stream=None):
    """fc2d_fft with the half spectrum [nf][nx][ld] complex128 (ld >= ny/2+1)."""
    import torch
    real = inp if direction == FC2D_FORWARD else out
    nf = _nf(real, grid)
    spec = out if direction == FC2D_FORWARD else inp
    if spec.dtype != torch.complex128 or spec.dim() != 3 or tuple(spec.shape[:2]) != (nf, grid.nx) or \
            spec.shape[2] < grid.ny // 2 + 1:
        raise ValueError("spectrum must be complex128 [nf][nx][ld] with ld >= ny/2+1")
    _check(_lib().fc2d_fft_ld(C.byref(grid), _dptr(inp, "in"), _dptr(out, "out"), int(direction),
                              int(spec.shape[2]), nf, _stream(stream)))


def fc2d_extend_fft_noalloc(plan, f_grid, f_bdry, work, spec, stream=None):
    """fc2d_extend_fft with its work space in the library's fixed scratch: allocates nothing."""
    _check(_lib().fc2d_extend_fft_noalloc(*_extend_fft_args(plan, f_grid, f_bdry, work, spec), _stream(stream)))


def fc2d_fft(grid, inp, out, direction, stream=None):
    import torch
    real = inp if direction == FC2D_FORWARD else out
    nf = _nf(real, grid)
    spec = out if direction == FC2D_FORWARD else inp
    if spec.dtype != torch.complex128 or spec.numel() != nf * grid.nx * (grid.ny // 2 + 1):
        raise ValueError("spectrum must be complex128 [nf][nx][ny/2+1]")
    _check(_lib().fc2d_fft(C.byref(grid), _dptr(inp, "in"), _dptr(out, "out"), int(direction), nf, _stream(stream)))


def fc2d_poisson_nodes(plan, nb):
    """Nystrom nodes q(2 pi j / nb), host array [nb, 2]."""
    xy = np.zeros((int(nb), 2))
    _check(_lib().fc2d_poisson_nodes(plan.handle, int(nb), C.c_void_p(xy.ctypes.data)))
    return xy


def fc2d_poisson_solve(plan, f_grid, f_bdry, g_nodes, u, stream=None):
    """Full Poisson solve; g_nodes [nf, nb] at fc2d_poisson_nodes(plan, nb).
    Returns the GMRES iterations summed over the fields."""
    import torch
    nf = _nf(f_grid, plan.grid)
    nb = g_nodes.shape[-1]
    if ((f_bdry is not None and f_bdry.numel() != nf * plan.info.n_bdry) or u.numel() != f_grid.numel()
            or g_nodes.numel() != nf * nb):
        raise ValueError("f_bdry / g_nodes / u sizes do not match the plan")
    it = C.c_int()
    _check(_lib().fc2d_poisson_solve(plan.handle, _dptr(f_grid, "f_grid", torch.float64),
                                     _bptr(plan, f_bdry), _dptr(g_nodes, "g_nodes", torch.float64),
                                     int(nb), _dptr(u, "u", torch.float64), nf, _stream(stream), C.byref(it)))
    return it.value


def _nspec(t, grid, name):
    import torch
    ns = grid.nx * (grid.ny // 2 + 1)
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or t.numel() % ns:
        raise ValueError("%s must be complex128 [nf][nx][ny/2+1]" % name)
    return t.numel() // ns


def fc2d_spectral_apply(grid, op, inp, out, stream=None):
    nf = _nspec(inp, grid, "in")
    if _nspec(out, grid, "out") != nf:
        raise ValueError("in and out hold different numbers of spectra")
    _check(_lib().fc2d_spectral_apply(C.byref(grid), int(op), _dptr(inp, "in"), _dptr(out, "out"), nf, _stream(stream)))


def ff_propagate(grid, c, t, u0h, u1h, uh, uth, stream=None):
    nf = _nspec(u0h, grid, "u0h")
    if any(_nspec(x, grid, n) != nf for x, n in ((u1h, "u1h"), (uh, "uh"), (uth, "uth"))):
        raise ValueError("u0h, u1h, uh and uth hold different numbers of spectra")
    _check(_lib().ff_propagate(C.byref(grid), float(c), float(t), _dptr(u0h, "u0h"), _dptr(u1h, "u1h"),
                               _dptr(uh, "uh"), _dptr(uth, "uth"), nf, _stream(stream)))


def fc2d_boundary_values(plan, u, f_bdry, stream=None):
    import torch
    nf = _nf(u, plan.grid)
    if f_bdry.numel() != nf * plan.info.n_bdry:
        raise ValueError("f_bdry size does not match the plan")
    _check(_lib().fc2d_boundary_values(plan.handle, _dptr(u, "u", torch.float64), _dptr(f_bdry, "f_bdry", torch.float64),
                                       nf, _stream(stream)))


class Batch:
    """Owning wrapper of fc2d_batch* (keeps its plans alive)."""

    def __init__(self, plans, nf, autotune=False, fused_ff=False, transposed=False, stream=None):
        self.plans = list(plans)
        arr = (C.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        nfa = (C.c_int * len(self.plans))(*[int(n) for n in nf])
        self.nf = [int(n) for n in nf]
        h = C.c_void_p()
        flags = ((FC2D_BATCH_AUTOTUNE if autotune else 0) | (FC2D_BATCH_FUSED_FF if fused_ff else 0)
                 | (FC2D_BATCH_TRANSPOSED if transposed else 0))
        _check(_lib().fc2d_batch_create(arr, nfa, len(self.plans), flags,
                                        _stream(stream), C.byref(h)))
        self._h = h

    def state(self, k):
        """(u, u_t) of plan k as torch tensors viewing the batch's device memory."""
        import torch
        u = C.c_void_p()
        ut = C.c_void_p()
        _check(_lib().fc2d_batch_state(self._h, int(k), C.byref(u), C.byref(ut)))
        g = self.plans[k].grid
        n = self.nf[k] * g.nx * g.ny
        return _view_device(u.value, n, (self.nf[k], g.nx, g.ny)), _view_device(ut.value, n, (self.nf[k], g.nx, g.ny))

    def info(self):
        pts = C.c_int64()
        nl = C.c_int()
        sf = C.c_int()
        _check(_lib().fc2d_batch_info(self._h, C.byref(pts), C.byref(nl), C.byref(sf)))
        return pts.value, nl.value, sf.value

    def run_ff(self, c, dt, steps, use_graph=True, stream=None):
        _check(_lib().fc2d_batch_run_ff(self._h, float(c), float(dt), int(steps), 1 if use_graph else 0,
                                        _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib().fc2d_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _view_device(ptr, n, shape):
    """A float64 torch tensor over library-owned device memory (no copy)."""
    import torch

    class _Arr:
        __cuda_array_interface__ = {"shape": (n,), "typestr": "<f8", "data": (ptr, False), "version": 2}

    return torch.as_tensor(_Arr(), device="cuda:0").view(*shape)


def fc2d_tune_set(knob, n, value):
    _check(_lib().fc2d_tune_set(int(knob), int(n), int(value)))


def fc2d_tune_get(knob, n=0):
    v = C.c_int()
    _check(_lib().fc2d_tune_get(int(knob), int(n), C.byref(v)))
    return v.value


def fc2d_trace_begin(stream=None):
    _check(_lib().fc2d_trace_begin(_stream(stream)))


def fc2d_trace_end(cap=4096):
    """Close the trace; returns [(kernel name, milliseconds)] in launch order."""
    n = C.c_int()
    names = (C.c_char_p * cap)()
    ms = (C.c_float * cap)()
    _check(_lib().fc2d_trace_end(C.byref(n), names, ms, cap))
    return [(names[i].decode(), float(ms[i])) for i in range(n.value)]


def fc2d_mlp_make_data(curves, cidx, theta, eta, width, X, Y, foot=None, iters=None, stream=None):
    """Training pairs: curves [ncurves][1 + 2 nmodes] float64, cidx [n] int32,
    theta / eta [n] float64 (device) -> X [n][8], Y [n][2] float32, foot [n][2]
    float64, iters [n] int32 (device, optional)."""
    import torch
    ncurves, ncoef = curves.shape
    n = cidx.numel()
    if X.numel() != n * FC2D_MLP_NIN or Y.numel() != 2 * n or theta.numel() != n or eta.numel() != n:
        raise ValueError("training-data array sizes disagree")
    _check(_lib().fc2d_mlp_make_data(_dptr(curves, "curves", torch.float64), int(ncurves), (int(ncoef) - 1) // 2,
                                     _dptr(cidx, "cidx", torch.int32), _dptr(theta, "theta", torch.float64),
                                     _dptr(eta, "eta", torch.float64), int(n), float(width),
                                     _dptr(X, "X", torch.float32), _dptr(Y, "Y", torch.float32),
                                     _dptr(foot, "foot", torch.float64) if foot is not None else None,
                                     _dptr(iters, "iters", torch.int32) if iters is not None else None,
                                     _stream(stream)))


def fc2d_mlp_forward(weights, X, out, stream=None):
    import torch
    n = X.numel() // FC2D_MLP_NIN
    if out.numel() != 2 * n or weights.numel() != FC2D_MLP_NW:
        raise ValueError("forward array sizes disagree")
    _check(_lib().fc2d_mlp_forward(_dptr(weights, "weights", torch.float32), _dptr(X, "X", torch.float32), int(n),
                                   _dptr(out, "out", torch.float32), _stream(stream)))


def fc2d_mlp_loss_grad(weights, X, Y, grad=None, loss=None, stream=None):
    import torch
    n = X.numel() // FC2D_MLP_NIN
    if Y.numel() != 2 * n or weights.numel() != FC2D_MLP_NW:
        raise ValueError("loss/gradient array sizes disagree")
    _check(_lib().fc2d_mlp_loss_grad(_dptr(weights, "weights", torch.float32), _dptr(X, "X", torch.float32),
                                     _dptr(Y, "Y", torch.float32), int(n),
                                     _dptr(grad, "grad", torch.float32) if grad is not None else None,
                                     _dptr(loss, "loss", torch.float32) if loss is not None else None,
                                     _stream(stream)))


def fc2d_mlp_train(weights, adam_m, adam_v, X, Y, batch, steps, t0, lr0, lr_min, t_total, loss_hist=None,
                   stream=None):
    import torch
    n = X.numel() // FC2D_MLP_NIN
    if Y.numel() != 2 * n or weights.numel() != FC2D_MLP_NW or adam_m.numel() != FC2D_MLP_NW or \
            adam_v.numel() != FC2D_MLP_NW or (loss_hist is not None and loss_hist.numel() < steps):
        raise ValueError("training array sizes disagree")
    _check(_lib().fc2d_mlp_train(_dptr(weights, "weights", torch.float32), _dptr(adam_m, "adam_m", torch.float32),
                                 _dptr(adam_v, "adam_v", torch.float32), _dptr(X, "X", torch.float32),
                                 _dptr(Y, "Y", torch.float32), int(n), int(batch), int(steps), int(t0),
                                 float(lr0), float(lr_min), int(t_total),
                                 _dptr(loss_hist, "loss_hist", torch.float32) if loss_hist is not None else None,
                                 _stream(stream)))


def fc2d_version():
    return _lib().fc2d_version()


FFR_OUT, FFR_INT, FFR_STEP, FFR_BND = 0, 1, 2, 3


class FF:
    """Owning wrapper of fc2d_ff* (Fourier Forwarding solver; keeps its plan alive)."""

    def __init__(self, plan, c=1.0, n_c=6, closure_nodes=0, stream=None):
        self.plan = plan
        h = C.c_void_p()
        _check(_lib().fc2d_ff_create(plan.handle, float(c), int(n_c), int(closure_nodes), _stream(stream),
                                     C.byref(h)))
        self._h = h
        info = fc2d_ff_info()
        _check(_lib().fc2d_ff_get_info(h, C.byref(info)))
        self.info = info

    def crossings(self):
        n = C.c_int64()
        _check(_lib().fc2d_ff_crossings(self._h, C.byref(n), None))
        xy = np.zeros((n.value, 2))
        _check(_lib().fc2d_ff_crossings(self._h, C.byref(n), C.c_void_p(xy.ctypes.data)))
        return xy

    def regions(self):
        g = self.plan.grid
        out = np.zeros((g.nx, g.ny), dtype=np.int8)
        _check(_lib().fc2d_ff_regions(self._h, C.c_void_p(out.ctypes.data)))
        return out

    def advance(self, u, ut, fb_u, fb_ut, bc_u, bc_ut, nsmall=None, stream=None):
        """Advance (u, ut) in place by nsmall small steps (default: one large step).
        fb_u, fb_ut [n_bdry]; bc_u, bc_ut [nsmall + 1][n_cross] (device float64)."""
        import torch
        g = self.plan.grid
        ns = self.info.K if nsmall is None else int(nsmall)
        nc = self.info.n_cross
        _check_out(u, "u", g.nx * g.ny, torch.float64)
        _check_out(ut, "ut", g.nx * g.ny, torch.float64)
        _check_out(fb_u, "fb_u", self.plan.info.n_bdry, torch.float64)
        _check_out(fb_ut, "fb_ut", self.plan.info.n_bdry, torch.float64)
        _check_out(bc_u, "bc_u", (ns + 1) * nc, torch.float64)
        _check_out(bc_ut, "bc_ut", (ns + 1) * nc, torch.float64)
        _check(_lib().fc2d_ff_advance(self._h, _dptr(u, "u"), _dptr(ut, "ut"), _dptr(fb_u, "fb_u"),
                                      _dptr(fb_ut, "fb_ut"), _dptr(bc_u, "bc_u"), _dptr(bc_ut, "bc_ut"), ns,
                                      _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _lib().fc2d_ff_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
