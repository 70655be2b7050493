"""Thin Python binding of ``libscitv.so`` (the C ABI declared in include/scitv.h).

Argument marshalling only: every function here checks tensor shapes, dtypes
and devices, allocates outputs with torch when the caller passes none, and
hands raw device pointers plus the current torch stream to the C function of
the same name. All computation happens in the library's HIP kernels; there is
no fallback. Importing this module raises if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscitv.so")

SCI_OK = 0
SCI_NOT_CONVERGED = 1
SCI_ERR_INVALID_ARG = -1
SCI_ERR_ALIAS = -2
SCI_ERR_NOMEM = -3
SCI_ERR_HIP = -4
SCI_ERR_UNSUPPORTED = -5

TV = {"atv": 0, "itv2d": 1, "vtv": 2}
DUAL = {"f32": 0, "bf16": 1, "f16": 2}
DUAL_TORCH = {0: torch.float32, 1: torch.bfloat16, 2: torch.float16}
SCHED = {"auto": 0, "stream": 1, "fused": 2}


class SciError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libscitv status {status}: {msg}")
        self.status = status


class sci_dims(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("B", ctypes.c_int32)]


class sci_tv_params(ctypes.Structure):
    _fields_ = [("tv", ctypes.c_int32), ("lambda_", ctypes.c_float), ("n_inner", ctypes.c_int32),
                ("accel", ctypes.c_int32), ("dual_dtype", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("gap_tol", ctypes.c_double), ("n_inner_max", ctypes.c_int32), ("gap_check_every", ctypes.c_int32),
                ("tile_shape", ctypes.c_int32), ("tile_passes", ctypes.c_int32), ("chambolle04", ctypes.c_int32),
                ("clip", ctypes.c_int32), ("clip_alpha", ctypes.c_float)]


class sci_solver_params(ctypes.Structure):
    _fields_ = [("tv", sci_tv_params), ("outer_iters", ctypes.c_int32), ("rho", ctypes.c_float),
                ("warm_dual", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("twist_alpha", ctypes.c_float),
                ("twist_beta", ctypes.c_float)]


class sci_problem(ctypes.Structure):
    _fields_ = [("d", sci_dims), ("Y", ctypes.c_void_p), ("C", ctypes.c_void_p), ("X_out", ctypes.c_void_p),
                ("Theta_out", ctypes.c_void_p), ("outer_iters", ctypes.c_int32)]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    V, I, P = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER
    D = sci_dims
    sig = {
        "sci_create": (I, [P(V), I]),
        "sci_destroy": (None, [V]),
        "sci_status_string": (ctypes.c_char_p, [I]),
        "sci_last_error": (ctypes.c_char_p, [V]),
        "sci_forward": (I, [V, D, V, V, V, V]),
        "sci_adjoint": (I, [V, D, V, V, V, V]),
        "sci_tv_denoise": (I, [V, D, P(sci_tv_params), V, V, V, V, P(ctypes.c_double), P(ctypes.c_int32), V]),
        "sci_gap_tv": (I, [V, D, P(sci_solver_params), V, V, V, V, V, V]),
        "sci_gap_tv_noalloc": (I, [V, D, P(sci_solver_params), V, V, V, V, V, V]),
        "sci_admm_tv": (I, [V, D, P(sci_solver_params), V, V, V, V, V, V]),
        "sci_fista_tv": (I, [V, D, P(sci_solver_params), V, V, V, V, V, V]),
        "sci_twist_tv": (I, [V, D, P(sci_solver_params), V, V, V, V, V, V]),
        "sci_psnr": (I, [V, ctypes.c_int64, V, V, ctypes.c_double, P(ctypes.c_double), V]),
        "sci_residual_sq": (I, [V, D, V, V, V, P(ctypes.c_double), V]),
        "sci_dual_gap": (I, [V, D, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, V, V, P(ctypes.c_double),
                             P(ctypes.c_double), V]),
        "sci_profile_enable": (I, [V, I]),
        "sci_wsnet_create": (I, [V, ctypes.c_int32, ctypes.c_int32, P(V)]),
        "sci_wsnet_destroy": (None, [V]),
        "sci_wsnet_param_count": (ctypes.c_int64, []),
        "sci_wsnet_set_loss": (I, [V, V, ctypes.c_int32]),
        "sci_wsnet_set_params": (I, [V, V, P(ctypes.c_float), ctypes.c_int64]),
        "sci_wsnet_get_params": (I, [V, V, P(ctypes.c_float), ctypes.c_int64]),
        "sci_wsnet_forward": (I, [V, V, D, V, V, V, ctypes.c_int32, V, V]),
        "sci_wsnet_grads": (I, [V, V, D, V, V, V, P(ctypes.c_float), P(ctypes.c_double), V]),
        "sci_wsnet_train_step": (I, [V, V, D, V, V, V, ctypes.c_float, P(ctypes.c_double), V]),
        "sci_gap_tv_adaptive": (I, [V, D, P(sci_solver_params), V, V, V, V, V, V, P(ctypes.c_int32),
                                    P(ctypes.c_int32), P(ctypes.c_int32), V]),
        "sci_gap_tv_batched": (I, [V, ctypes.c_int32, P(sci_problem), P(sci_solver_params), V]),
        "sci_autotune_batched": (I, [V, ctypes.c_int32, P(sci_problem), P(sci_solver_params), P(ctypes.c_int32),
                                     P(ctypes.c_double), V]),
        "sci_tile_shape_count": (I, []),
        "sci_tile_shape_info": (I, [ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32)]),
        "sci_tile_shape_pipelined": (I, [ctypes.c_int32]),
        "sci_autotune": (I, [V, D, P(sci_tv_params), V, P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_double),
                             V]),
        "sci_profile_read": (I, [V, ctypes.c_char_p, P(ctypes.c_int64), P(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = load_library()


# ---- marshalling helpers ------------------------------------------------------

def _stream(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _dev(t: Optional[torch.Tensor], dtype=torch.float32, shape=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device (cuda) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _check(ctx, status: int, allow=(SCI_OK,)):
    if status in allow:
        return status
    msg = lib.sci_last_error(ctx).decode() if ctx else ""
    base = lib.sci_status_string(status).decode()
    raise SciError(status, f"{base}: {msg}" if msg else base)


def _dims(vol: torch.Tensor) -> sci_dims:
    if vol.dim() != 3:
        raise ValueError("video tensors are [B][nx][ny]")
    B, nx, ny = vol.shape
    return sci_dims(nx, ny, B)


def tv_params(tv="atv", lam=0.1, n_inner=5, accel=True, dual_dtype="f32", schedule="auto", gap_tol=0.0,
              n_inner_max=0, gap_check_every=0, tile_shape=0, tile_passes=0, chambolle04=False, clip=False,
              clip_alpha=0.0) -> sci_tv_params:
    return sci_tv_params(TV[tv] if isinstance(tv, str) else int(tv), float(lam), int(n_inner), int(bool(accel)),
                         DUAL[dual_dtype] if isinstance(dual_dtype, str) else int(dual_dtype),
                         SCHED[schedule] if isinstance(schedule, str) else int(schedule), float(gap_tol),
                         int(n_inner_max), int(gap_check_every), int(tile_shape), int(tile_passes),
                         int(bool(chambolle04)), int(bool(clip)), float(clip_alpha))


def solver_params(outer_iters=50, rho=0.0, warm_dual=False, use_graph=False, twist_alpha=0.0, twist_beta=0.0,
                  **tv) -> sci_solver_params:
    return sci_solver_params(tv_params(**tv), int(outer_iters), float(rho), int(bool(warm_dual)),
                             int(bool(use_graph)), float(twist_alpha), float(twist_beta))


# ---- entry points (same names as the C ABI) ---------------------------------------

def sci_create(device: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(None, lib.sci_create(ctypes.byref(h), int(device)))
    return h


def sci_destroy(ctx) -> None:
    lib.sci_destroy(ctx)


def sci_forward(ctx, C: torch.Tensor, X: torch.Tensor, Y: Optional[torch.Tensor] = None, stream=None):
    d = _dims(C)
    if Y is None:
        Y = torch.empty((d.nx, d.ny), device=C.device, dtype=torch.float32)
    _check(ctx, lib.sci_forward(ctx, d, _dev(C, name="C"), _dev(X, shape=C.shape, name="X"),
                                _dev(Y, shape=(d.nx, d.ny), name="Y"), _stream(stream)))
    return Y


def sci_adjoint(ctx, C: torch.Tensor, Y: torch.Tensor, X: Optional[torch.Tensor] = None, stream=None):
    d = _dims(C)
    if X is None:
        X = torch.empty_like(C)
    _check(ctx, lib.sci_adjoint(ctx, d, _dev(C, name="C"), _dev(Y, shape=(d.nx, d.ny), name="Y"),
                                _dev(X, shape=C.shape, name="X"), _stream(stream)))
    return X


def sci_tv_denoise(ctx, X_in: torch.Tensor, params: sci_tv_params, Theta_out=None, dual_init=None, dual_out=None,
                   want_gap: bool = False, stream=None):
    """Returns (theta, rel_gap or None, iterations, status)."""
    d = _dims(X_in)
    if Theta_out is None:
        Theta_out = torch.empty_like(X_in)
    dshape = (2,) + tuple(X_in.shape)
    ddt = DUAL_TORCH[params.dual_dtype]
    gap = ctypes.c_double(0.0)
    its = ctypes.c_int32(0)
    st = lib.sci_tv_denoise(ctx, d, ctypes.byref(params), _dev(X_in, name="X_in"),
                            _dev(Theta_out, shape=X_in.shape, name="Theta_out"),
                            _dev(dual_init, ddt, dshape, "dual_init"), _dev(dual_out, ddt, dshape, "dual_out"),
                            ctypes.byref(gap) if want_gap else None, ctypes.byref(its), _stream(stream))
    _check(ctx, st, allow=(SCI_OK, SCI_NOT_CONVERGED))
    return Theta_out, (gap.value if want_gap else None), its.value, st


def _outer(fn, ctx, Y, C, params, X_out, Theta_out, X_init, stream):
    d = _dims(C)
    if X_out is None:
        X_out = torch.empty_like(C)
    _check(ctx, fn(ctx, d, ctypes.byref(params), _dev(Y, shape=(d.nx, d.ny), name="Y"), _dev(C, name="C"),
                   _dev(X_out, shape=C.shape, name="X_out"), _dev(Theta_out, shape=C.shape, name="Theta_out"),
                   _dev(X_init, shape=C.shape, name="X_init"), _stream(stream)))
    return X_out, Theta_out


def sci_gap_tv(ctx, Y, C, params: sci_solver_params, X_out=None, Theta_out=None, X_init=None, stream=None):
    """GAP-TV; returns (X_out, Theta_out)."""
    return _outer(lib.sci_gap_tv, ctx, Y, C, params, X_out, Theta_out, X_init, stream)


def sci_gap_tv_noalloc(ctx, Y, C, params: sci_solver_params, X_out, Theta_out, X_init=None, stream=None):
    """GAP-TV without any device allocation by the library (caller-owned
    X_out and Theta_out); returns (X_out, Theta_out)."""
    return _outer(lib.sci_gap_tv_noalloc, ctx, Y, C, params, X_out, Theta_out, X_init, stream)


def sci_admm_tv(ctx, Y, C, params: sci_solver_params, X_out=None, Theta_out=None, X_init=None, stream=None):
    """ADMM-TV; returns (X_out, Theta_out)."""
    return _outer(lib.sci_admm_tv, ctx, Y, C, params, X_out, Theta_out, X_init, stream)


def sci_fista_tv(ctx, Y, C, params: sci_solver_params, X_out=None, Theta_out=None, X_init=None, stream=None):
    """FISTA-TV; returns (X_out, Theta_out)."""
    return _outer(lib.sci_fista_tv, ctx, Y, C, params, X_out, Theta_out, X_init, stream)


def sci_twist_tv(ctx, Y, C, params: sci_solver_params, X_out=None, Theta_out=None, X_init=None, stream=None):
    """TwIST-TV; returns (X_out, Theta_out)."""
    return _outer(lib.sci_twist_tv, ctx, Y, C, params, X_out, Theta_out, X_init, stream)


def _problems(items):
    """items: sequence of dicts with Y, C, X_out, optional Theta_out, optional outer_iters."""
    arr = (sci_problem * len(items))()
    for k, it in enumerate(items):
        C = it["C"]
        d = _dims(C)
        arr[k] = sci_problem(d, _dev(it["Y"], shape=(d.nx, d.ny), name="Y"), _dev(C, name="C"),
                             _dev(it["X_out"], shape=C.shape, name="X_out"),
                             _dev(it.get("Theta_out"), shape=C.shape, name="Theta_out"), int(it.get("outer_iters", 0)))
    return arr


def sci_gap_tv_batched(ctx, items, params: sci_solver_params, stream=None):
    """GAP-TV for a list of measurements (dicts with Y, C, X_out[, Theta_out, outer_iters])."""
    arr = _problems(items)
    _check(ctx, lib.sci_gap_tv_batched(ctx, len(items), arr, ctypes.byref(params), _stream(stream)))


def sci_autotune_batched(ctx, items, params: sci_solver_params, stream=None):
    """Returns (best 1-based tile shape, [ms per shape]) for the batched denoise launch."""
    arr = _problems(items)
    n = lib.sci_tile_shape_count()
    best = ctypes.c_int32(0)
    times = (ctypes.c_double * n)()
    _check(ctx, lib.sci_autotune_batched(ctx, len(items), arr, ctypes.byref(params), ctypes.byref(best), times,
                                         _stream(stream)))
    return best.value, list(times)


def sci_psnr(ctx, a: torch.Tensor, ref: torch.Tensor, peak: float = 1.0, stream=None) -> float:
    if a.shape != ref.shape:
        raise ValueError("psnr: shape mismatch")
    out = ctypes.c_double(0.0)
    _check(ctx, lib.sci_psnr(ctx, a.numel(), _dev(a, name="a"), _dev(ref, name="ref"), float(peak),
                             ctypes.byref(out), _stream(stream)))
    return out.value


def sci_residual_sq(ctx, C, X, Y, stream=None) -> float:
    d = _dims(C)
    out = ctypes.c_double(0.0)
    _check(ctx, lib.sci_residual_sq(ctx, d, _dev(C, name="C"), _dev(X, shape=C.shape, name="X"),
                                    _dev(Y, shape=(d.nx, d.ny), name="Y"), ctypes.byref(out), _stream(stream)))
    return out.value


def sci_dual_gap(ctx, X, p, tv="atv", lam=0.1, stream=None):
    """(gap, primal) of the denoising problem at dual p (dtype picks the storage type)."""
    d = _dims(X)
    dt = {torch.float32: 0, torch.bfloat16: 1, torch.float16: 2}[p.dtype]
    g, pr = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(ctx, lib.sci_dual_gap(ctx, d, TV[tv] if isinstance(tv, str) else int(tv), dt, float(lam),
                                 _dev(X, name="X"), _dev(p, p.dtype, (2,) + tuple(X.shape), "p"), ctypes.byref(g),
                                 ctypes.byref(pr), _stream(stream)))
    return g.value, pr.value


def sci_tile_shape_count() -> int:
    return lib.sci_tile_shape_count()


def sci_tile_shape_info(shape: int):
    """(rows per wavefront, wavefronts per workgroup, columns per lane) of a 1-based shape."""
    r, w, c = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    _check(None, lib.sci_tile_shape_info(int(shape), ctypes.byref(r), ctypes.byref(w), ctypes.byref(c)))
    return r.value, w.value, c.value


def sci_tile_shape_pipelined(shape: int) -> bool:
    """True for a row-pipelined shape, False for a tiled one (1-based)."""
    v = lib.sci_tile_shape_pipelined(int(shape))
    _check(None, min(v, 0))
    return v == 1


def sci_autotune(ctx, X: torch.Tensor, params: sci_tv_params, stream=None):
    """Time every fused (tile shape, pass count) on X; returns (best 1-based
    shape, best pass count, [[ms per pass-count candidate] per shape])."""
    n = lib.sci_tile_shape_count()
    best, passes = ctypes.c_int32(0), ctypes.c_int32(0)
    times = (ctypes.c_double * (3 * n))()
    _check(ctx, lib.sci_autotune(ctx, _dims(X), ctypes.byref(params), _dev(X, name="X"), ctypes.byref(best),
                                 ctypes.byref(passes), times, _stream(stream)))
    t = list(times)
    return best.value, passes.value, [t[3 * k:3 * k + 3] for k in range(n)]


def sci_profile_enable(ctx, enable: bool = True) -> None:
    _check(ctx, lib.sci_profile_enable(ctx, int(bool(enable))))


def sci_profile_read(ctx, family: str):
    """(launches, total milliseconds) recorded for a kernel family."""
    n, ms = ctypes.c_int64(0), ctypes.c_double(0.0)
    _check(ctx, lib.sci_profile_read(ctx, family.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


# ---- learned warm start -----------------------------------------------------------

def sci_wsnet_create(ctx, c_in: int = 1, c_out: int = 2):
    h = ctypes.c_void_p()
    _check(ctx, lib.sci_wsnet_create(ctx, int(c_in), int(c_out), ctypes.byref(h)))
    return h


def sci_wsnet_destroy(net) -> None:
    lib.sci_wsnet_destroy(net)


def sci_wsnet_param_count() -> int:
    return lib.sci_wsnet_param_count()


WSNET_LOSS = {"dual": 0, "theta": 1}


def sci_wsnet_set_loss(ctx, net, kind) -> None:
    """Training loss of the network: "dual" (MSE over the dual channels) or
    "theta" (mean of (D^T r)^2 over the voxels)."""
    _check(ctx, lib.sci_wsnet_set_loss(ctx, net, WSNET_LOSS[kind] if isinstance(kind, str) else int(kind)))


def sci_wsnet_set_params(ctx, net, params) -> None:
    import numpy as np
    a = np.ascontiguousarray(params, dtype=np.float32).ravel()
    _check(ctx, lib.sci_wsnet_set_params(ctx, net, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))


def sci_wsnet_get_params(ctx, net):
    import numpy as np
    a = np.empty(lib.sci_wsnet_param_count(), dtype=np.float32)
    _check(ctx, lib.sci_wsnet_get_params(ctx, net, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))
    return a


def sci_wsnet_forward(ctx, net, X, tv="itv2d", base=None, want_raw=False, want_dual=True, stream=None, c_out=2):
    """(raw output [c_out][B][nx][ny] or None, projected dual [2][B][nx][ny] or
    None); c_out is the network's output channel count."""
    d = _dims(X)
    raw = torch.empty((c_out,) + tuple(X.shape), device=X.device) if want_raw else None
    dual = torch.empty((2,) + tuple(X.shape), device=X.device) if want_dual else None
    _check(ctx, lib.sci_wsnet_forward(ctx, net, d, _dev(X, name="X"), _dev(base, shape=(2,) + tuple(X.shape), name="base"),
                                      _dev(raw, name="raw"),
                                      TV[tv] if isinstance(tv, str) else int(tv), _dev(dual, name="dual"),
                                      _stream(stream)))
    return raw, dual


def sci_wsnet_grads(ctx, net, X, target, base=None, stream=None):
    """(loss, gradient in the padded parameter layout)."""
    import numpy as np
    d = _dims(X)
    g = np.empty(lib.sci_wsnet_param_count(), dtype=np.float32)
    loss = ctypes.c_double(0.0)
    _check(ctx, lib.sci_wsnet_grads(ctx, net, d, _dev(X, name="X"), _dev(base, name="base"),
                                    _dev(target, name="target"),
                                    g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(loss),
                                    _stream(stream)))
    return loss.value, g


def sci_wsnet_train_step(ctx, net, X, target, lr, base=None, want_loss=True, stream=None):
    d = _dims(X)
    loss = ctypes.c_double(0.0)
    _check(ctx, lib.sci_wsnet_train_step(ctx, net, d, _dev(X, name="X"), _dev(base, name="base"),
                                         _dev(target, name="target"), float(lr),
                                         ctypes.byref(loss) if want_loss else None, _stream(stream)))
    return loss.value if want_loss else None


def sci_gap_tv_adaptive(ctx, Y, C, params: sci_solver_params, net=None, X_out=None, Theta_out=None, X_init=None,
                        stream=None):
    """Gap-controlled GAP-TV; returns (X_out, total inner iterations, fallbacks,
    calls started from the network's prediction)."""
    d = _dims(C)
    if X_out is None:
        X_out = torch.empty_like(C)
    its, fb, ns = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    _check(ctx, lib.sci_gap_tv_adaptive(ctx, d, ctypes.byref(params), _dev(Y, shape=(d.nx, d.ny), name="Y"),
                                        _dev(C, name="C"), _dev(X_out, shape=C.shape, name="X_out"),
                                        _dev(Theta_out, shape=C.shape, name="Theta_out"),
                                        _dev(X_init, shape=C.shape, name="X_init"), net, ctypes.byref(its),
                                        ctypes.byref(fb), ctypes.byref(ns), _stream(stream)))
    return X_out, its.value, fb.value, ns.value


class Context:
    """Owns one sci_ctx on a device; frees it on close()/garbage collection."""

    def __init__(self, device: int = 0):
        self.handle = sci_create(device)

    def close(self):
        if self.handle is not None and self.handle.value:
            sci_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
