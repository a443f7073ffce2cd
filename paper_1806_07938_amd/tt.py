"""Thin Python binding of the C ABI in include/tt.h (argument marshalling only).

Every step of the reconstructor runs in the HIP library libtt.so; this module
only converts Python arguments to the C structs, passes device pointers of
PyTorch tensors (PyTorch supplies device memory and the stream) and turns
status codes into exceptions.  If the library is not built, importing the
library raises: there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import math
import os
import sys
import weakref
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtt.so")

TT_OK, TT_INVALID_ARG, TT_HIP_ERROR, TT_OUT_OF_MEMORY, TT_NOT_CONVERGED, TT_BREAKDOWN, TT_NOT_READY = range(7)
PREC_F32, PREC_F64, PREC_F16, PREC_BF16 = 0, 1, 2, 3
PRECOND_NONE, PRECOND_CIRCULANT, PRECOND_LEARNED = 0, 1, 2
METHOD_CG, METHOD_MINRES = 0, 1
SOLVER_PERSISTENT, SOLVER_KERNELS, SOLVER_BATCHED = 0, 1, 2
MODEL_HUDGIN, MODEL_FRIED = 0, 1

# Every function declared in include/tt.h.
EXPORTED = (
    "tt_create", "tt_destroy", "tt_generate_kernels", "tt_kernels_destroy", "tt_kernels_copy",
    "tt_set_system", "tt_set_noise_xy", "tt_set_mode_removal", "tt_get_system_info", "tt_matvec", "tt_matvec_f64", "tt_matvec_batch",
    "tt_matvec_noalloc", "tt_matvec_batch_prec", "tt_create_view", "tt_tune_batch", "tt_learned_create", "tt_learned_destroy", "tt_learned_weight_count",
    "tt_learned_get_weights", "tt_learned_set_weights", "tt_learned_apply", "tt_learned_train_step",
    "tt_learned_train", "tt_set_learned",
    "tt_solve_frame", "tt_solve_batch", "tt_project", "tt_status_string", "tt_last_error", "tt_pupil_mask",
)


class TTError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_status_name(status)}: {msg}")
        self.status = status


class _Geometry(C.Structure):
    _fields_ = [("n", C.c_int), ("n_gs", C.c_int), ("pad_L", C.c_int), ("gradient_model", C.c_int),
                ("D", C.c_double), ("h_lgs", C.c_double), ("gs_xy", C.POINTER(C.c_double)),
                ("valid", C.POINTER(C.c_ubyte)), ("obstruction", C.c_double)]


class _Atmosphere(C.Structure):
    _fields_ = [("n_layer", C.c_int), ("h", C.POINTER(C.c_double)), ("w", C.POINTER(C.c_double)),
                ("r0", C.c_double), ("L0", C.c_double)]


class _Target(C.Structure):
    _fields_ = [("beta_x", C.c_double), ("beta_y", C.c_double), ("n_prime", C.c_int), ("pad_L", C.c_int)]


class _SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("precision", C.c_int), ("solver", C.c_int),
                ("refine_drop", C.c_double), ("preconditioner", C.c_int), ("method", C.c_int),
                ("graph", C.c_int)]


class _SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("refinements", C.c_int), ("status", C.c_int),
                ("rel_residual", C.c_double), ("recursive_residual", C.c_double),
                ("kernel_ms", C.c_double), ("kernel_launches", C.c_int), ("fallback", C.c_int)]


class _SystemInfo(C.Structure):
    _fields_ = [("n", C.c_int), ("n_gs", C.c_int), ("pad_L", C.c_int), ("n_vs", C.c_int), ("n_slopes", C.c_int),
                ("n_vphi", C.c_int), ("n_prime", C.c_int), ("proj_pad_L", C.c_int), ("n_layer", C.c_int),
                ("spectra_bytes_f32", C.c_size_t), ("spectra_bytes_f64", C.c_size_t),
                ("proj_spectra_bytes", C.c_size_t)]


class _TrainOpts(C.Structure):
    _fields_ = [("n_pairs", C.c_int), ("steps", C.c_int), ("batch", C.c_int), ("lr", C.c_double)]


class _TrainInfo(C.Structure):
    _fields_ = [("objective_first", C.c_double), ("objective_last", C.c_double), ("ms", C.c_double)]


_lib = None

# Library handles still open.  They are closed by an exit hook registered after
# torch has initialised the device (exit hooks run last-registered first, so
# before torch's own teardown and before the HIP runtime's static destructors);
# a handle found open during interpreter finalisation is left to the process
# exit instead of calling into HIP from a finaliser.
_open_handles = weakref.WeakSet()
_exit_hook = False


def _close_open_handles():
    # views before the contexts they share a system with
    for h in sorted(list(_open_handles), key=lambda o: 0 if getattr(o, "_base", None) is not None else 1):
        try:
            h.close()
        except Exception:
            pass


def close_all():
    """Close every library handle still open (contexts and kernel tables)."""
    _close_open_handles()


def _track(obj):
    global _exit_hook
    _open_handles.add(obj)
    if not _exit_hook:
        atexit.register(_close_open_handles)
        _exit_hook = True


def load(path: str = LIB_PATH):
    """Load libtt.so (once).  Raises RuntimeError if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_1806_07938_amd.build`")
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.tt_create.argtypes = [C.POINTER(vp), C.c_int, vp]
    lib.tt_destroy.argtypes = [vp]
    lib.tt_create_view.argtypes = [C.POINTER(vp), vp, vp]
    lib.tt_tune_batch.argtypes = [C.POINTER(vp), C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_float)]
    lib.tt_generate_kernels.argtypes = [vp, C.POINTER(_Geometry), C.POINTER(_Atmosphere), C.POINTER(vp)]
    lib.tt_kernels_destroy.argtypes = [vp]
    lib.tt_kernels_copy.argtypes = [vp, C.POINTER(C.c_double), C.c_size_t]
    lib.tt_set_system.argtypes = [vp, vp, C.POINTER(C.c_double), C.c_double, C.POINTER(_Target)]
    lib.tt_get_system_info.argtypes = [vp, C.POINTER(_SystemInfo)]
    lib.tt_set_noise_xy.argtypes = [vp, C.POINTER(C.c_double)]
    lib.tt_set_mode_removal.argtypes = [vp, C.c_int]
    lib.tt_matvec.argtypes = [vp, vp, vp]
    lib.tt_matvec_f64.argtypes = [vp, vp, vp]
    lib.tt_matvec_noalloc.argtypes = [vp, vp, vp]
    lib.tt_matvec_batch_prec.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(vp), C.POINTER(vp), C.c_int, C.c_int,
                                         C.POINTER(C.c_float)]
    lib.tt_learned_create.argtypes = [C.POINTER(vp), C.c_int, C.c_int, C.c_int, C.c_ulonglong]
    lib.tt_learned_destroy.argtypes = [vp]
    lib.tt_learned_weight_count.argtypes = [vp, C.POINTER(C.c_size_t)]
    lib.tt_learned_get_weights.argtypes = [vp, C.POINTER(C.c_float), C.c_size_t]
    lib.tt_learned_set_weights.argtypes = [vp, C.POINTER(C.c_float), C.c_size_t]
    lib.tt_learned_apply.argtypes = [vp, vp, vp, vp]
    lib.tt_learned_train_step.argtypes = [vp, vp, vp, vp, C.c_int, C.c_double, C.POINTER(C.c_double),
                                          C.POINTER(C.c_double)]
    lib.tt_learned_train.argtypes = [vp, C.POINTER(vp), C.c_int, C.POINTER(_TrainOpts), C.POINTER(_TrainInfo)]
    lib.tt_set_learned.argtypes = [vp, vp]
    lib.tt_solve_frame.argtypes = [vp, vp, vp, vp, vp, C.POINTER(_SolveOpts), C.POINTER(_SolveInfo)]
    lib.tt_project.argtypes = [vp, vp, vp]
    lib.tt_solve_batch.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                   C.POINTER(vp), C.POINTER(_SolveOpts), C.POINTER(_SolveInfo)]
    lib.tt_pupil_mask.argtypes = [C.c_int, C.c_double, C.c_double, C.POINTER(C.c_ubyte), C.POINTER(C.c_int)]
    lib.tt_status_string.argtypes = [C.c_int]
    lib.tt_status_string.restype = C.c_char_p
    lib.tt_last_error.argtypes = []
    lib.tt_last_error.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("tt_status_string", "tt_last_error"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _status_name(s: int) -> str:
    try:
        return load().tt_status_string(s).decode()
    except Exception:
        return f"status {s}"


def _check(status: int, allow=(TT_OK,)):
    if status not in allow:
        raise TTError(status, load().tt_last_error().decode())
    return status


def _dptr(t, dtype, numel: Optional[int] = None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {dtype} tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


@dataclass
class SolveInfo:
    iterations: int
    refinements: int
    status: int
    rel_residual: float
    recursive_residual: float
    kernel_ms: float = 0.0
    kernel_launches: int = 0
    fallback: int = -1


class Kernels:
    """Generated FP64 covariance tables (owned by the library)."""

    def __init__(self, handle, n, n_gs):
        self._h = handle
        self.n, self.n_gs = n, n_gs
        _track(self)

    @property
    def count(self):
        return self.n_gs * (self.n_gs + 1) // 2 * 3 * (2 * self.n - 1) ** 2

    def tables(self) -> np.ndarray:
        """(pairs, 3, 2n-1, 2n-1) array: pairs (g, h), g <= h row-major; xx, xy, yy;
        [v + n-1, u + n-1] with u the column lag and v the row lag."""
        out = np.empty(self.count, dtype=np.float64)
        _check(load().tt_kernels_copy(self._h, out.ctypes.data_as(C.POINTER(C.c_double)), out.size))
        m = 2 * self.n - 1
        return out.reshape(-1, 3, m, m)

    def close(self):
        if self._h:
            load().tt_kernels_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Context:
    """One library context bound to a device and a stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        lib = load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream_obj = stream
        sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        h = C.c_void_p()
        _check(lib.tt_create(C.byref(h), device, C.c_void_p(sp)))
        self._h = h
        self.device = device
        self._keep = []
        _track(self)

    # -- set-up -----------------------------------------------------------
    def generate_kernels(self, n: int, n_gs: int, pad_L: int, D: float, h_lgs: float,
                         gs_xy: Sequence[Sequence[float]], valid, h, w, r0: float, L0: float,
                         model: int = MODEL_HUDGIN, obstruction: float = 0.0) -> Kernels:
        """valid None: the library's valid-subaperture rule with `obstruction`."""
        gs = np.ascontiguousarray(np.asarray(gs_xy, dtype=np.float64).reshape(-1))
        vp = None
        if valid is not None:
            vm = np.ascontiguousarray(np.asarray(valid, dtype=np.uint8).reshape(-1))
            vp = vm.ctypes.data_as(C.POINTER(C.c_ubyte))
        hh = np.ascontiguousarray(np.asarray(h, dtype=np.float64))
        ww = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
        geo = _Geometry(n, n_gs, pad_L, int(model), float(D), float(h_lgs) if math.isfinite(h_lgs) else math.inf,
                        gs.ctypes.data_as(C.POINTER(C.c_double)), vp, float(obstruction))
        atm = _Atmosphere(hh.size, hh.ctypes.data_as(C.POINTER(C.c_double)),
                          ww.ctypes.data_as(C.POINTER(C.c_double)), float(r0), float(L0))
        out = C.c_void_p()
        _check(load().tt_generate_kernels(self._h, C.byref(geo), C.byref(atm), C.byref(out)))
        return Kernels(out, n, n_gs)

    def set_system(self, kernels: Kernels, noise_scalar: float = 0.0, noise_var=None,
                   target: Optional[tuple] = None, n_prime: int = 0, proj_pad_L: int = 0):
        nv = None
        if noise_var is not None:
            arr = np.ascontiguousarray(np.asarray(noise_var, dtype=np.float64))
            self._keep = [arr]
            nv = arr.ctypes.data_as(C.POINTER(C.c_double))
        tgt = None
        if target is not None:
            tgt = C.byref(_Target(float(target[0]), float(target[1]), int(n_prime), int(proj_pad_L)))
        _check(load().tt_set_system(self._h, kernels._h, nv, float(noise_scalar), tgt))
        self.info = self.system_info()

    def set_noise_xy(self, cov_xy=None):
        """2x2 noise blocks (elongated LGS spots): cov_xy (n_gs, n_vs) x-y noise
        covariances, or None to remove them."""
        p = None
        if cov_xy is not None:
            arr = np.ascontiguousarray(np.asarray(cov_xy, dtype=np.float64).reshape(-1))
            self._keep_xy = arr
            p = arr.ctypes.data_as(C.POINTER(C.c_double))
        _check(load().tt_set_noise_xy(self._h, p))

    def set_mode_removal(self, on: bool = True):
        """Tip/tilt/focus removal M_s (and M_phi on the projection), §2.F."""
        _check(load().tt_set_mode_removal(self._h, 1 if on else 0))

    def system_info(self) -> dict:
        s = _SystemInfo()
        _check(load().tt_get_system_info(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in _SystemInfo._fields_}

    # -- hot path ---------------------------------------------------------
    def matvec(self, x, y=None):
        import torch
        n = self.info["n_slopes"]
        if y is None:
            y = torch.empty(n, dtype=torch.float32, device=x.device)
        _check(load().tt_matvec(self._h, _dptr(x, torch.float32, n), _dptr(y, torch.float32, n)))
        return y

    def matvec_noalloc(self, x, y):
        """tt_matvec_noalloc: the product of matvec without any device allocation
        (work buffers in the library's fixed per-device array); y is required."""
        import torch
        n = self.info["n_slopes"]
        _check(load().tt_matvec_noalloc(self._h, _dptr(x, torch.float32, n), _dptr(y, torch.float32, n)))
        return y

    def matvec_f64(self, x, y=None):
        import torch
        n = self.info["n_slopes"]
        if y is None:
            y = torch.empty(n, dtype=torch.float64, device=x.device)
        _check(load().tt_matvec_f64(self._h, _dptr(x, torch.float64, n), _dptr(y, torch.float64, n)))
        return y

    def solve(self, s, x0=None, zeta=None, phi=None, project: bool = True, tol: float = 1e-6,
              max_iter: int = 20000, precision: int = PREC_F32, solver: int = SOLVER_PERSISTENT,
              refine_drop: float = 1e-3, preconditioner: int = PRECOND_NONE, method: int = METHOD_CG,
              allow=(TT_OK,), graph: bool = False):
        """Solve for zeta (float64) and, if a target is set and project, phi (float32)."""
        import torch
        n = self.info["n_slopes"]
        if zeta is None:
            zeta = torch.empty(n, dtype=torch.float64, device=s.device)
        pphi = None
        if project and self.info["n_vphi"] > 0:
            if phi is None:
                phi = torch.empty(self.info["n_vphi"], dtype=torch.float32, device=s.device)
            pphi = _dptr(phi, torch.float32, self.info["n_vphi"])
        else:
            phi = None
        opts = _SolveOpts(float(tol), int(max_iter), int(precision), int(solver), float(refine_drop),
                          int(preconditioner), int(method), 1 if graph else 0)
        inf = _SolveInfo()
        px0 = _dptr(x0, torch.float64, n) if x0 is not None else None
        st = load().tt_solve_frame(self._h, _dptr(s, torch.float32, n), px0, _dptr(zeta, torch.float64, n),
                                   pphi, C.byref(opts), C.byref(inf))
        _check(st, allow=allow)
        return zeta, phi, SolveInfo(inf.iterations, inf.refinements, inf.status, inf.rel_residual,
                                    inf.recursive_residual, inf.kernel_ms, inf.kernel_launches, inf.fallback)

    def view(self, stream=None):
        """tt_create_view: a context sharing this one's system, with its own
        stream (default: torch's current stream) and solver buffers."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        h = C.c_void_p()
        _check(load().tt_create_view(C.byref(h), self._h, C.c_void_p(sp)))
        v = Context.__new__(Context)
        v._h, v.device, v._keep, v._stream_obj, v._base = h, self.device, [], stream, self
        v.info = dict(self.info, n_vphi=0, n_prime=0, proj_pad_L=0)
        _track(v)
        return v

    def set_learned(self, net):
        """Attach (or with None detach) the network of TT_PRECOND_LEARNED solves."""
        _check(load().tt_set_learned(self._h, net._h if net is not None else None))
        self._learned = net

    def project(self, zeta, phi=None):
        import torch
        n = self.info["n_slopes"]
        if phi is None:
            phi = torch.empty(self.info["n_vphi"], dtype=torch.float32, device=zeta.device)
        _check(load().tt_project(self._h, _dptr(zeta, torch.float64, n), _dptr(phi, torch.float32, self.info["n_vphi"])))
        return phi

    def close(self):
        if getattr(self, "_h", None):
            _check(load().tt_destroy(self._h))
            self._h = None
            self._base = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Learned:
    """A learned preconditioner P = K^T K (tt_learned_*)."""

    def __init__(self, n_gs: int, hidden: int = 32, seed: int = 1806, device: int = 0):
        h = C.c_void_p()
        _check(load().tt_learned_create(C.byref(h), int(device), int(n_gs), int(hidden), C.c_ulonglong(seed)))
        self._h = h
        self.n_gs, self.hidden = n_gs, hidden
        cnt = C.c_size_t()
        _check(load().tt_learned_weight_count(self._h, C.byref(cnt)))
        self.count = cnt.value
        _track(self)

    def layer_shapes(self):
        Cc, H = 2 * self.n_gs, self.hidden
        return [(H, Cc, 3, 3), (H, H, 3, 3), (H, H, 3, 3), (Cc, H, 3, 3)]

    def weights(self):
        """FP32 master weights as four (out, in, 3, 3) arrays."""
        out = np.empty(self.count, dtype=np.float32)
        _check(load().tt_learned_get_weights(self._h, out.ctypes.data_as(C.POINTER(C.c_float)), out.size))
        ws, o = [], 0
        for shp in self.layer_shapes():
            k = int(np.prod(shp))
            ws.append(out[o:o + k].reshape(shp).copy())
            o += k
        return ws

    def set_weights(self, ws):
        flat = np.ascontiguousarray(np.concatenate([np.asarray(w, dtype=np.float32).ravel() for w in ws]))
        _check(load().tt_learned_set_weights(self._h, flat.ctypes.data_as(C.POINTER(C.c_float)), flat.size))

    def apply(self, ctx, r, z=None):
        import torch
        n = ctx.info["n_slopes"]
        if z is None:
            z = torch.empty(n, dtype=torch.float32, device=r.device)
        _check(load().tt_learned_apply(self._h, ctx._h, _dptr(r, torch.float32, n), _dptr(z, torch.float32, n)))
        return z

    def train_step(self, ctx, R, E, lr: float):
        """One step on device pairs R, E (batch, n_slopes) float32; returns (J, t)
        at the weights used."""
        import torch
        n = ctx.info["n_slopes"]
        assert R.shape == E.shape and R.shape[1] == n
        J, t = C.c_double(), C.c_double()
        _check(load().tt_learned_train_step(self._h, ctx._h, _dptr(R, torch.float32), _dptr(E, torch.float32),
                                            int(R.shape[0]), float(lr), C.byref(J), C.byref(t)))
        return J.value, t.value

    def train(self, contexts, n_pairs: int = 20000, steps: int = 3000, batch: int = 16, lr: float = 3e-3):
        """tt_learned_train over contexts sharing a geometry; returns the info dict."""
        m = len(contexts)
        arr = (C.c_void_p * m)(*[c._h for c in contexts])
        opts = _TrainOpts(int(n_pairs), int(steps), int(batch), float(lr))
        inf = _TrainInfo()
        _check(load().tt_learned_train(self._h, arr, m, C.byref(opts), C.byref(inf)))
        return {"objective_first": inf.objective_first, "objective_last": inf.objective_last, "ms": inf.ms}

    def close(self):
        if getattr(self, "_h", None):
            load().tt_learned_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def pupil_mask(n: int, D: float, obstruction: float) -> np.ndarray:
    """tt_pupil_mask: the library's valid-subaperture rule, (n, n) bool (host only)."""
    out = np.zeros(n * n, dtype=np.uint8)
    cnt = C.c_int()
    _check(load().tt_pupil_mask(int(n), float(D), float(obstruction), out.ctypes.data_as(C.POINTER(C.c_ubyte)),
                                C.byref(cnt)))
    m = out.reshape(n, n).astype(bool)
    assert int(m.sum()) == cnt.value
    return m


def system_from(ctx: Context, wl, target: bool = True, pad_L: Optional[int] = None, proj_pad_L: int = 0,
                n_prime: int = 0) -> Kernels:
    """Generate kernels and set the system of `ctx` from any object with the
    attributes n, D, gs, h_lgs, h, w, r0, L0, valid, pad_L, noise_var, target."""
    model = MODEL_FRIED if getattr(wl, "model", "hudgin") == "fried" else MODEL_HUDGIN
    k = ctx.generate_kernels(wl.n, wl.gs.shape[0], int(pad_L or wl.pad_L), wl.D, wl.h_lgs, wl.gs, wl.valid,
                             wl.h, wl.w, wl.r0, wl.L0, model=model)
    ctx.set_system(k, noise_scalar=wl.noise_var, target=(tuple(wl.target) if target else None),
                   n_prime=n_prime, proj_pad_L=proj_pad_L)
    return k


def matvec_batch(contexts, xs, ys=None, timing: bool = False, precision: int = PREC_F32, split: int = 0):
    """tt_matvec_batch: ys[i] = A_i xs[i] (device float32 vectors) for every
    context in one call on the stream of contexts[0] (tt_matvec_batch_prec with
    the spectra in FP16 / BF16 storage for those precisions).  With timing=True
    the call waits and also returns the three phase durations in ms."""
    import torch
    m = len(contexts)
    assert len(xs) == m
    if ys is None:
        ys = [torch.empty(c.info["n_slopes"], dtype=torch.float32, device=x.device) for c, x in zip(contexts, xs)]
    arr = C.c_void_p * max(m, 1)
    hs = arr(*[c._h for c in contexts])
    xp = arr(*[_dptr(x, torch.float32, c.info["n_slopes"]) for c, x in zip(contexts, xs)])
    yp = arr(*[_dptr(y, torch.float32, c.info["n_slopes"]) for c, y in zip(contexts, ys)])
    ms = (C.c_float * 3)()
    if precision == PREC_F32 and not split:
        _check(load().tt_matvec_batch(hs, m, xp, yp, ms if timing else None))
    else:
        _check(load().tt_matvec_batch_prec(hs, m, xp, yp, int(precision), int(split), ms if timing else None))
    return (ys, [float(v) for v in ms]) if timing else ys


def tune_batch(contexts, op: int = 0, precision: int = PREC_F32):
    """tt_tune_batch: choose the batched column kernel's frequency split for this
    batch; returns (best split, {split: mean ms per call or None})."""
    m = len(contexts)
    hs = (C.c_void_p * m)(*[c._h for c in contexts])
    best = C.c_int()
    ms = (C.c_float * 3)()
    _check(load().tt_tune_batch(hs, m, int(op), int(precision), C.byref(best), ms))
    return best.value, {s: (float(v) if v > 0 else None) for s, v in zip((1, 2, 4), ms)}


def solve_batch(contexts, slopes, tol: float = 1e-6, max_iter: int = 20000, precision: int = PREC_F32,
                solver: int = SOLVER_PERSISTENT, refine_drop: float = 1e-3, preconditioner: int = PRECOND_NONE,
                method: int = METHOD_CG, allow=(TT_OK,), graph: bool = False):
    """tt_solve_batch: frame i (device float32 slopes) on contexts[i]; returns
    (zetas, phis, infos, status).  phis[i] is None without a target."""
    import torch
    m = len(contexts)
    assert len(slopes) == m
    zetas, phis, sp, zp, pp = [], [], [], [], []
    for ctx, s in zip(contexts, slopes):
        n = ctx.info["n_slopes"]
        z = torch.empty(n, dtype=torch.float64, device=s.device)
        zetas.append(z)
        sp.append(_dptr(s, torch.float32, n))
        zp.append(_dptr(z, torch.float64, n))
        if ctx.info["n_vphi"] > 0:
            ph = torch.empty(ctx.info["n_vphi"], dtype=torch.float32, device=s.device)
            phis.append(ph)
            pp.append(_dptr(ph, torch.float32, ctx.info["n_vphi"]))
        else:
            phis.append(None)
            pp.append(None)
    arr = C.c_void_p * max(m, 1)
    hs = arr(*[c._h for c in contexts])
    opts = _SolveOpts(float(tol), int(max_iter), int(precision), int(solver), float(refine_drop),
                      int(preconditioner), int(method), 1 if graph else 0)
    infos = (_SolveInfo * max(m, 1))()
    use_phi = all(p is not None for p in pp) and m > 0
    st = load().tt_solve_batch(hs, m, arr(*sp), None, arr(*zp), arr(*pp) if use_phi else None, C.byref(opts), infos)
    _check(st, allow=allow)
    out = [SolveInfo(i.iterations, i.refinements, i.status, i.rel_residual, i.recursive_residual, i.kernel_ms,
                     i.kernel_launches, i.fallback) for i in list(infos)[:m]]
    return zetas, (phis if use_phi else [None] * m), out, st
