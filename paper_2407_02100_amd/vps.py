"""Thin ctypes binding of libvps (the C ABI declared in include/vps.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Torch tensors supply device memory (``data_ptr``) and the HIP
stream (``torch.cuda.current_stream().cuda_stream``).  The module-level
functions carry the C names; :class:`Context` wraps a ``vps_context*``.

Loading fails loudly (``VpsError``) when ``libvps.so`` has not been built;
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvps.so")

VPS_OK, VPS_E_ARG, VPS_E_UNSUPPORTED, VPS_E_HIP = 0, -1, -2, -3
VPS_E_NOMEM, VPS_E_NOT_CONVERGED, VPS_E_NONFINITE, VPS_E_STATE = -4, -5, -6, -7
VPS_F64, VPS_F32 = 0, 1
VPS_COEF_CONST, VPS_COEF_CELL_MEAN_FDM, VPS_COEF_CELL_LEARNED, VPS_COEF_CELL_EXACT = 0, 1, 2, 3

_COEF = {"const": VPS_COEF_CONST, "mean": VPS_COEF_CELL_MEAN_FDM, "learned": VPS_COEF_CELL_LEARNED,
         "exact": VPS_COEF_CELL_EXACT}
_ALGORITHM = {"combined": 0, "separated": 1}
_DTYPE = {"f64": VPS_F64, "f32": VPS_F32}


class VpsError(RuntimeError):
    def __init__(self, status, message=""):
        self.status = status
        super().__init__(f"{status_string(status)} ({status}): {message}" if message else status_string(status))


class vps_config(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("degree", ctypes.c_int), ("n_cells", ctypes.c_int),
                ("n_levels", ctypes.c_int), ("pre_sweeps", ctypes.c_int), ("post_sweeps", ctypes.c_int),
                ("vcycle_dtype", ctypes.c_int), ("coef", ctypes.c_int), ("patches_per_block", ctypes.c_int),
                ("stream_min_cells", ctypes.c_int), ("algorithm", ctypes.c_int), ("patch_order", ctypes.c_int),
                ("batch_layers", ctypes.c_int), ("patches_per_wave", ctypes.c_int),
                ("vcycle_graph", ctypes.c_int), ("wave_rows_2d", ctypes.c_int)]


class vps_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual_true", ctypes.c_double),
                ("seconds", ctypes.c_double), ("fallback_patches", ctypes.c_longlong)]


VPS_MAX_LEVELS = 16


class vps_timing(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int),
                ("smooth_s", ctypes.c_double * VPS_MAX_LEVELS),
                ("smooth_sweeps", ctypes.c_longlong * VPS_MAX_LEVELS),
                ("residual_s", ctypes.c_double * VPS_MAX_LEVELS),
                ("restrict_s", ctypes.c_double * VPS_MAX_LEVELS),
                ("prolong_s", ctypes.c_double * VPS_MAX_LEVELS),
                ("coarse_s", ctypes.c_double), ("cg_operator_s", ctypes.c_double),
                ("cg_vector_s", ctypes.c_double), ("vcycles", ctypes.c_longlong)]


_vp = ctypes.c_void_p
_i = ctypes.c_int
_ll = ctypes.c_longlong
_d = ctypes.c_double
_f = ctypes.c_float

# name -> (restype, argtypes)
SIGNATURES = {
    "vps_create": (_i, [ctypes.POINTER(vps_config), _vp, ctypes.POINTER(_vp)]),
    "vps_destroy": (_i, [_vp]),
    "vps_set_stream": (_i, [_vp, _vp]),
    "vps_level_nodes": (ctypes.c_size_t, [_vp, _i]),
    "vps_level_cells": (_i, [_vp, _i]),
    "vps_level_patches": (_ll, [_vp, _i]),
    "vps_set_coefficient": (_i, [_vp, _vp]),
    "vps_set_patch_scaling": (_i, [_vp, _i, _vp]),
    "vps_apply": (_i, [_vp, _i, _vp, _vp, _i]),
    "vps_residual": (_i, [_vp, _i, _vp, _vp, _vp, _i]),
    "vps_restrict": (_i, [_vp, _i, _vp, _vp, _i]),
    "vps_prolongate_add": (_i, [_vp, _i, _vp, _vp, _i]),
    "vps_coarse_solve": (_i, [_vp, _vp, _vp, _i]),
    "vps_smooth_color": (_i, [_vp, _i, _vp, _vp, _i, _i]),
    "vps_smooth": (_i, [_vp, _i, _vp, _vp, _i, _i, _i]),
    "vps_vcycle": (_i, [_vp, _vp, _vp]),
    "vps_solve": (_i, [_vp, _vp, _vp, _d, _i, ctypes.POINTER(vps_solve_info)]),
    "vps_vcycle_iterate": (_i, [_vp, _vp, _vp, _i, ctypes.POINTER(_d)]),
    "vps_patch_features": (_i, [_vp, _i, _vp]),
    "vps_patch_rho8": (_i, [_vp, _i, _vp]),
    "vps_rho8_features": (_i, [_vp, _vp, _ll, _vp]),
    "vps_patch_targets": (_i, [_vp, _vp, _ll, _vp, _vp]),
    "vps_mlp_forward": (_i, [_vp, _vp, _vp, _ll, _vp, _vp]),
    "vps_mlp_loss_grad": (_i, [_vp, _vp, _vp, _ll, _vp, _vp]),
    "vps_mlp_backward": (_i, [_vp, _vp, _vp, _vp, _vp, _ll, _vp]),
    "vps_mlp_backward_noalloc": (_i, [_vp, _vp, _vp, _vp, _vp, _ll, _vp]),
    "vps_mlp_adam": (_i, [_vp, _vp, _vp, _vp, _vp, _i, _f, _f, _f, _f]),
    "vps_mlp_infer_patches": (_i, [_vp, _i, _vp, ctypes.POINTER(_ll)]),
    "vps_timing_enable": (_i, [_vp, _i]),
    "vps_timing_get": (_i, [_vp, ctypes.POINTER(vps_timing)]),
    "vps_sync": (_i, [_vp]),
    "vps_status_string": (ctypes.c_char_p, [_i]),
    "vps_last_error": (ctypes.c_char_p, [_vp]),
}

_lib = None


def lib():
    """The loaded libvps.so (raises VpsError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise VpsError(VPS_E_STATE, f"{LIB_PATH} is missing; build it with "
                                        "`python -m paper_2407_02100_amd.build`")
        # torch ships its own HIP/HSA runtime (same SONAMEs as /opt/rocm's);
        # importing it first makes libvps bind to that one, so the process
        # holds a single runtime and torch's stream handles are valid here.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().vps_status_string(int(s)).decode()


def _ptr(t):
    """Device pointer of a contiguous CUDA tensor (or None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise VpsError(VPS_E_ARG, "tensor must live on the GPU")
    if not t.is_contiguous():
        raise VpsError(VPS_E_ARG, "tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _dtype_of(t):
    import torch
    if t.dtype == torch.float64:
        return VPS_F64
    if t.dtype == torch.float32:
        return VPS_F32
    raise VpsError(VPS_E_ARG, f"unsupported dtype {t.dtype}")


def _check_args(what, specs, same_dtype=False):
    """Host-side checks before any call into the library: dtype, element count, then one CUDA device.

    specs: (name, tensor or None, dtype name 'f64'/'f32'/None, element count or None).  A pointer the
    library reads or writes covers exactly the elements the C ABI documents, so a wrong dtype or size
    would make a kernel access memory outside the tensor; these are rejected here with VPS_E_ARG.
    """
    import torch
    want = {"f64": torch.float64, "f32": torch.float32}
    seen = []
    for name, t, dt, numel in specs:
        if t is None:
            continue
        if not isinstance(t, torch.Tensor):
            raise VpsError(VPS_E_ARG, f"{what}: {name} must be a torch tensor")
        if dt is not None and t.dtype != want[dt]:
            raise VpsError(VPS_E_ARG, f"{what}: {name} must be {want[dt]}, got {t.dtype}")
        if t.dtype not in (torch.float64, torch.float32):
            raise VpsError(VPS_E_ARG, f"{what}: {name} has unsupported dtype {t.dtype}")
        if numel is not None and t.numel() != numel:
            raise VpsError(VPS_E_ARG, f"{what}: {name} must have {numel} elements, got {t.numel()}")
        seen.append((name, t))
    if same_dtype and len({t.dtype for _, t in seen}) > 1:
        raise VpsError(VPS_E_ARG, f"{what}: " + ", ".join(f"{n} {t.dtype}" for n, t in seen)
                       + " must share one dtype")
    devs = set()
    for name, t in seen:
        if not t.is_cuda:
            raise VpsError(VPS_E_ARG, f"{what}: {name} must live on the GPU")
        if not t.is_contiguous():
            raise VpsError(VPS_E_ARG, f"{what}: {name} must be contiguous")
        devs.add(t.device)
    if len(devs) > 1:
        raise VpsError(VPS_E_ARG, f"{what}: tensors on several devices {sorted(map(str, devs))}")


def _current_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """Owns a vps_context*.  Methods mirror the C entry points (without the prefix)."""

    def __init__(self, dim, degree, n_cells, n_levels, pre=1, post=1, vcycle_dtype="f64",
                 coef="const", patches_per_block=0, stream=None, stream_min_cells=0, algorithm="combined",
                 patch_order=0, batch_layers=0, patches_per_wave=0, vcycle_graph=False, wave_rows_2d=0):
        cfg = vps_config(dim, degree, n_cells, n_levels, pre, post, _DTYPE[vcycle_dtype], _COEF[coef],
                         patches_per_block, stream_min_cells, _ALGORITHM[algorithm], patch_order, batch_layers,
                         patches_per_wave, int(bool(vcycle_graph)),
                         wave_rows_2d)
        self.cfg = cfg
        self._shape(dim, degree, n_cells, n_levels)
        h = _vp()
        st = lib().vps_create(ctypes.byref(cfg), stream if stream is not None else _current_stream(),
                              ctypes.byref(h))
        if st != VPS_OK:
            raise VpsError(st, lib().vps_last_error(None).decode())
        self.h = h

    # -- helpers --
    def _shape(self, dim, degree, n_cells, n_levels):
        """Element counts the C ABI documents per level (host arithmetic on the configuration only)."""
        self.dim, self.degree, self.n_levels = dim, degree, n_levels
        self.h = None
        cells = [max(n_cells >> (n_levels - 1 - l), 0) for l in range(n_levels)]
        self._cells = cells
        self._nodes = [(degree * c + 1) ** dim for c in cells]
        self._patches = [max(c - 1, 0) ** dim for c in cells]
        self._nin = 2 ** dim
        self._nout = (2 * degree - 1) ** dim
        self._nparams = mlp_param_count(self._nin, self._nout)

    def _level(self, what, level, lo=0):
        if not (lo <= level < self.n_levels):
            raise VpsError(VPS_E_ARG, f"{what}: level {level} outside [{lo}, {self.n_levels})")
        return level

    def _check(self, st, what):
        if st != VPS_OK:
            msg = lib().vps_last_error(self.h).decode() if self.h else ""
            raise VpsError(st, f"{what}: {msg}")

    def close(self):
        if getattr(self, "h", None):
            lib().vps_destroy(self.h)
            self.h = None

    destroy = close

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- queries --
    def level_nodes(self, level):
        return int(lib().vps_level_nodes(self.h, level))

    def level_cells(self, level):
        return int(lib().vps_level_cells(self.h, level))

    def level_patches(self, level):
        return int(lib().vps_level_patches(self.h, level))

    def set_stream(self, stream):
        self._check(lib().vps_set_stream(self.h, stream), "vps_set_stream")

    # -- set-up --
    def set_coefficient(self, rho_cells):
        _check_args("vps_set_coefficient", [("rho_cells", rho_cells, "f64", self._cells[-1] ** self.dim)])
        self._check(lib().vps_set_coefficient(self.h, _ptr(rho_cells)), "vps_set_coefficient")

    def set_patch_scaling(self, level, c):
        self._level("vps_set_patch_scaling", level)
        _check_args("vps_set_patch_scaling", [("c", c, "f32", self._patches[level] * self._nout)])
        self._check(lib().vps_set_patch_scaling(self.h, level, _ptr(c)), "vps_set_patch_scaling")

    # -- level operators --
    def apply(self, level, u, Au):
        n = self._nodes[self._level("vps_apply", level)]
        _check_args("vps_apply", [("u", u, None, n), ("Au", Au, None, n)], same_dtype=True)
        self._check(lib().vps_apply(self.h, level, _ptr(u), _ptr(Au), _dtype_of(u)), "vps_apply")

    def residual(self, level, b, u, r):
        n = self._nodes[self._level("vps_residual", level)]
        _check_args("vps_residual", [("b", b, None, n), ("u", u, None, n), ("r", r, None, n)], same_dtype=True)
        self._check(lib().vps_residual(self.h, level, _ptr(b), _ptr(u), _ptr(r), _dtype_of(u)), "vps_residual")

    def restrict(self, fine_level, r_fine, r_coarse):
        f = self._level("vps_restrict", fine_level, lo=1)
        _check_args("vps_restrict", [("r_fine", r_fine, None, self._nodes[f]),
                                     ("r_coarse", r_coarse, None, self._nodes[f - 1])], same_dtype=True)
        self._check(lib().vps_restrict(self.h, fine_level, _ptr(r_fine), _ptr(r_coarse), _dtype_of(r_fine)),
                    "vps_restrict")

    def prolongate_add(self, fine_level, e_coarse, u_fine):
        f = self._level("vps_prolongate_add", fine_level, lo=1)
        _check_args("vps_prolongate_add", [("e_coarse", e_coarse, None, self._nodes[f - 1]),
                                           ("u_fine", u_fine, None, self._nodes[f])], same_dtype=True)
        self._check(lib().vps_prolongate_add(self.h, fine_level, _ptr(e_coarse), _ptr(u_fine),
                                             _dtype_of(u_fine)), "vps_prolongate_add")

    def coarse_solve(self, b, x):
        _check_args("vps_coarse_solve", [("b", b, None, self._nodes[0]), ("x", x, None, self._nodes[0])],
                    same_dtype=True)
        self._check(lib().vps_coarse_solve(self.h, _ptr(b), _ptr(x), _dtype_of(b)), "vps_coarse_solve")

    # -- smoother --
    def smooth_color(self, level, u, b, color):
        n = self._nodes[self._level("vps_smooth_color", level)]
        _check_args("vps_smooth_color", [("u", u, None, n), ("b", b, None, n)], same_dtype=True)
        self._check(lib().vps_smooth_color(self.h, level, _ptr(u), _ptr(b), _dtype_of(u), color),
                    "vps_smooth_color")

    def smooth(self, level, u, b, sweeps=1, reverse=False):
        n = self._nodes[self._level("vps_smooth", level)]
        _check_args("vps_smooth", [("u", u, None, n), ("b", b, None, n)], same_dtype=True)
        self._check(lib().vps_smooth(self.h, level, _ptr(u), _ptr(b), _dtype_of(u), sweeps, int(reverse)),
                    "vps_smooth")

    # -- multigrid / solver --
    def vcycle(self, r, z):
        n = self._nodes[-1]
        _check_args("vps_vcycle", [("r", r, "f64", n), ("z", z, "f64", n)])
        self._check(lib().vps_vcycle(self.h, _ptr(r), _ptr(z)), "vps_vcycle")

    def solve(self, b, u, rtol=1e-10, maxit=100, check=True):
        n = self._nodes[-1]
        _check_args("vps_solve", [("b", b, "f64", n), ("u", u, "f64", n)])
        info = vps_solve_info()
        st = lib().vps_solve(self.h, _ptr(b), _ptr(u), rtol, maxit, ctypes.byref(info))
        if check:
            self._check(st, "vps_solve")
        return {"status": st, "iterations": info.iterations, "rel_residual_true": info.rel_residual_true,
                "seconds": info.seconds, "fallback_patches": info.fallback_patches}

    def vcycle_iterate(self, b, u, iters):
        n = self._nodes[-1]
        _check_args("vps_vcycle_iterate", [("b", b, "f64", n), ("u", u, "f64", n)])
        hist = (ctypes.c_double * (iters + 1))()
        self._check(lib().vps_vcycle_iterate(self.h, _ptr(b), _ptr(u), iters, hist), "vps_vcycle_iterate")
        return list(hist)

    # -- learned scaling --
    def patch_features(self, level, x):
        lv = self._level("vps_patch_features", level)
        _check_args("vps_patch_features", [("x", x, "f32", self._patches[lv] * self._nin)])
        self._check(lib().vps_patch_features(self.h, level, _ptr(x)), "vps_patch_features")

    def patch_rho8(self, level, rho8):
        lv = self._level("vps_patch_rho8", level)
        _check_args("vps_patch_rho8", [("rho8", rho8, "f64", self._patches[lv] * self._nin)])
        self._check(lib().vps_patch_rho8(self.h, level, _ptr(rho8)), "vps_patch_rho8")

    def rho8_features(self, rho8, x):
        n = rho8.shape[0]
        _check_args("vps_rho8_features", [("rho8", rho8, "f64", n * self._nin), ("x", x, "f32", n * self._nin)])
        self._check(lib().vps_rho8_features(self.h, _ptr(rho8), rho8.shape[0], _ptr(x)), "vps_rho8_features")

    def patch_targets(self, rho8, cstar, log_target=None):
        n = rho8.shape[0]
        _check_args("vps_patch_targets", [("rho8", rho8, "f64", n * self._nin), ("cstar", cstar, "f64", n * self._nout),
                                          ("log_target", log_target, "f32", n * self._nout)])
        self._check(lib().vps_patch_targets(self.h, _ptr(rho8), rho8.shape[0], _ptr(cstar), _ptr(log_target)),
                    "vps_patch_targets")

    def mlp_forward(self, params, x, y, act=None):
        n = x.shape[0]
        _check_args("vps_mlp_forward", [("params", params, "f32", self._nparams), ("x", x, "f32", n * self._nin),
                                        ("y", y, "f32", n * self._nout), ("act", act, "f32", n * 2 * 64)])
        self._check(lib().vps_mlp_forward(self.h, _ptr(params), _ptr(x), x.shape[0], _ptr(y), _ptr(act)),
                    "vps_mlp_forward")

    def mlp_loss_grad(self, y, t, dy, loss=None):
        n = y.shape[0]
        _check_args("vps_mlp_loss_grad", [("y", y, "f32", n * self._nout), ("t", t, "f32", n * self._nout),
                                          ("dy", dy, "f32", n * self._nout), ("loss", loss, "f32", 1)])
        self._check(lib().vps_mlp_loss_grad(self.h, _ptr(y), _ptr(t), y.shape[0], _ptr(dy), _ptr(loss)),
                    "vps_mlp_loss_grad")

    def mlp_backward(self, params, x, act, dy, dparams):
        n = x.shape[0]
        _check_args("vps_mlp_backward", [("params", params, "f32", self._nparams), ("x", x, "f32", n * self._nin),
                                         ("act", act, "f32", n * 2 * 64), ("dy", dy, "f32", n * self._nout),
                                         ("dparams", dparams, "f32", self._nparams)])
        self._check(lib().vps_mlp_backward(self.h, _ptr(params), _ptr(x), _ptr(act), _ptr(dy), x.shape[0],
                                           _ptr(dparams)), "vps_mlp_backward")

    def mlp_backward_noalloc(self, params, x, act, dy, dparams):
        n = x.shape[0]
        _check_args("vps_mlp_backward_noalloc", [("params", params, "f32", self._nparams),
                                                 ("x", x, "f32", n * self._nin), ("act", act, "f32", n * 2 * 64),
                                                 ("dy", dy, "f32", n * self._nout),
                                                 ("dparams", dparams, "f32", self._nparams)])
        self._check(lib().vps_mlp_backward_noalloc(self.h, _ptr(params), _ptr(x), _ptr(act), _ptr(dy), n,
                                                   _ptr(dparams)), "vps_mlp_backward_noalloc")

    def mlp_adam(self, params, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        P = self._nparams
        _check_args("vps_mlp_adam", [("params", params, "f32", P), ("g", g, "f32", P), ("m", m, "f32", P),
                                     ("v", v, "f32", P)])
        self._check(lib().vps_mlp_adam(self.h, _ptr(params), _ptr(g), _ptr(m), _ptr(v), step, lr, b1, b2, eps),
                    "vps_mlp_adam")

    def mlp_infer_patches(self, level, params):
        self._level("vps_mlp_infer_patches", level)
        _check_args("vps_mlp_infer_patches", [("params", params, "f32", self._nparams)])
        fb = ctypes.c_longlong(0)
        self._check(lib().vps_mlp_infer_patches(self.h, level, _ptr(params), ctypes.byref(fb)),
                    "vps_mlp_infer_patches")
        return int(fb.value)

    def timing_enable(self, enable=True):
        self._check(lib().vps_timing_enable(self.h, int(enable)), "vps_timing_enable")

    def timing_get(self):
        t = vps_timing()
        self._check(lib().vps_timing_get(self.h, ctypes.byref(t)), "vps_timing_get")
        L = t.n_levels
        return {"n_levels": L, "smooth_s": list(t.smooth_s[:L]), "smooth_sweeps": list(t.smooth_sweeps[:L]),
                "residual_s": list(t.residual_s[:L]), "restrict_s": list(t.restrict_s[:L]),
                "prolong_s": list(t.prolong_s[:L]), "coarse_s": t.coarse_s, "cg_operator_s": t.cg_operator_s,
                "cg_vector_s": t.cg_vector_s, "vcycles": t.vcycles}

    def sync(self):
        self._check(lib().vps_sync(self.h), "vps_sync")


def vps_create(*args, **kwargs) -> Context:
    return Context(*args, **kwargs)


def _method_alias(name):
    def f(ctx, *args, **kwargs):
        return getattr(ctx, name)(*args, **kwargs)
    f.__name__ = "vps_" + name
    f.__doc__ = f"Module-level form of Context.{name} (C entry point vps_{name})."
    return f


for _n in ("destroy", "set_stream", "level_nodes", "level_cells", "level_patches", "set_coefficient",
           "set_patch_scaling", "apply", "residual", "restrict", "prolongate_add", "coarse_solve",
           "smooth_color", "smooth", "vcycle", "solve", "vcycle_iterate", "patch_features", "patch_rho8",
           "rho8_features", "patch_targets",
           "mlp_forward", "mlp_loss_grad", "mlp_backward", "mlp_backward_noalloc", "mlp_adam", "mlp_infer_patches", "timing_enable",
           "timing_get", "sync"):
    globals()["vps_" + _n] = _method_alias(_n)


def vps_status_string(s):
    return status_string(s)


def mlp_param_count(nin, nout, hidden=64):
    return hidden * nin + hidden + hidden * hidden + hidden + nout * hidden + nout
