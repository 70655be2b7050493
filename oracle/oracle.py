"""Python view of the FP64 CPU oracle (``scitv_oracle.c``).

TEST INFRASTRUCTURE ONLY: the independent reference that the HIP library is
checked against. Only the tests, the package smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.

All functions take and return float64 numpy arrays (inputs are upcast); the
layouts are those of the C file: videos ``[B][nx][ny]``, images ``[nx][ny]``,
duals ``[2][B][nx][ny]``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "scitv_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

TV_KINDS = {"atv": 0, "itv2d": 1, "vtv": 2}

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (strict IEEE double, OpenMP for element-wise loops)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-ffp-contract=off", SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    lib = ctypes.CDLL(LIB)
    P = ctypes.POINTER(ctypes.c_double)
    i, d = ctypes.c_int, ctypes.c_double
    sig = {
        "orc_forward": (None, [i, i, i, P, P, P]),
        "orc_adjoint": (None, [i, i, i, P, P, P]),
        "orc_weights": (None, [i, i, i, P, d, P]),
        "orc_grad": (None, [i, i, i, P, P, P]),
        "orc_grad_adj": (None, [i, i, i, P, P, P]),
        "orc_tv_value": (d, [i, i, i, i, P]),
        "orc_project_dual": (None, [i, i, i, i, P, P]),
        "orc_fgp_beta": (None, [i, P]),
        "orc_tv_denoise": (i, [i, i, i, i, d, i, i, i, i, P, P, P, P, P]),
        "orc_dual_gap": (d, [i, i, i, i, d, P, P, P]),
        "orc_gap_tv": (i, [i, i, i, i, d, i, i, i, i, i, d, P, P, P, P, P]),
        "orc_admm_tv": (i, [i, i, i, i, d, d, i, i, i, i, i, d, P, P, P, P, P]),
        "orc_clip_denoise": (i, [i, i, i, d, d, i, P, P, P, P, P]),
        "orc_lipschitz": (d, [i, i, i, P]),
        "orc_fista_tv": (i, [i, i, i, i, d, i, i, i, i, P, P, P, P, P]),
        "orc_twist_tv": (i, [i, i, i, i, d, d, d, i, i, i, i, P, P, P, P, P]),
        "orc_psnr": (d, [ctypes.c_long, P, P, d]),
        "orc_residual_sq": (d, [i, i, i, P, P, P]),
        "orc_set_threads": (i, [i]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dims(vol):
    B, nx, ny = vol.shape
    return B, nx, ny


def _kind(tv) -> int:
    return TV_KINDS[tv] if isinstance(tv, str) else int(tv)


def forward(C, X):
    """Y = sum_k C_k * X_k (Eq. (3)/(4), without noise)."""
    C, X = _d(C), _d(X)
    B, nx, ny = _dims(X)
    Y = np.empty((nx, ny))
    _load().orc_forward(B, nx, ny, _p(C), _p(X), _p(Y))
    return Y


def adjoint(C, Y):
    """Phi^T Y: X_k = C_k * Y."""
    C, Y = _d(C), _d(Y)
    B, nx, ny = _dims(C)
    X = np.empty((B, nx, ny))
    _load().orc_adjoint(B, nx, ny, _p(C), _p(Y), _p(X))
    return X


def weights(C, rho=0.0):
    """Element-wise inverse of diag(Phi Phi^T) + rho (zero where not positive)."""
    C = _d(C)
    B, nx, ny = _dims(C)
    S = np.empty((nx, ny))
    _load().orc_weights(B, nx, ny, _p(C), float(rho), _p(S))
    return S


def grad(theta):
    """D theta -> dual-shaped [2][B][nx][ny] (Eq. (7), zero-padded)."""
    th = _d(theta)
    B, nx, ny = _dims(th)
    g = np.empty((2, B, nx, ny))
    _load().orc_grad(B, nx, ny, _p(th), _p(g[0]), _p(g[1]))
    return g


def grad_adj(p):
    """D^T p for a dual-shaped p."""
    p = _d(p)
    _, B, nx, ny = p.shape
    out = np.empty((B, nx, ny))
    _load().orc_grad_adj(B, nx, ny, _p(np.ascontiguousarray(p[0])), _p(np.ascontiguousarray(p[1])), _p(out))
    return out


def tv_value(theta, tv):
    th = _d(theta)
    B, nx, ny = _dims(th)
    return _load().orc_tv_value(_kind(tv), B, nx, ny, _p(th))


def project_dual(q, tv):
    q = _d(q).copy()
    _, B, nx, ny = q.shape
    h, v = np.ascontiguousarray(q[0]), np.ascontiguousarray(q[1])
    _load().orc_project_dual(_kind(tv), B, nx, ny, _p(h), _p(v))
    return np.stack([h, v])


def fgp_beta(n):
    b = np.empty(max(n, 0))
    if n > 0:
        _load().orc_fgp_beta(n, _p(b))
    return b


def tv_denoise(x, lam, n_iter, tv="atv", accel=True, p_init=None, chambolle04=False,
               literal_out=False, return_dual=False):
    """prox_{lam TV}(x) by FGP (accel) or Chambolle projected gradient, fixed n_iter."""
    x = _d(x)
    B, nx, ny = _dims(x)
    th = np.empty_like(x)
    pin = None if p_init is None else _d(p_init)
    ph = np.empty_like(x) if return_dual else None
    pv = np.empty_like(x) if return_dual else None
    _load().orc_tv_denoise(_kind(tv), B, nx, ny, float(lam), int(n_iter), int(bool(accel)),
                           int(bool(chambolle04)), int(bool(literal_out)), _p(x), _p(pin), _p(th),
                           _p(ph), _p(pv))
    if return_dual:
        return th, np.stack([ph, pv])
    return th


def dual_gap(x, p, lam, tv):
    """(gap, primal) of the denoising problem for the feasible dual p."""
    x, p = _d(x), _d(p)
    B, nx, ny = _dims(x)
    prim = ctypes.c_double(0.0)
    g = _load().orc_dual_gap(_kind(tv), B, nx, ny, float(lam), _p(x), _p(p), ctypes.byref(prim))
    return g, prim.value


def _variant(chambolle04, clip, tv):
    if clip:
        if _kind(tv) != 0:
            raise ValueError("ATV-Clip is defined for anisotropic TV only")
        return 2
    return 1 if chambolle04 else 0


def gap_tv(Y, C, lam, T, N, tv="atv", accel=True, x_init=None, warm_dual=False, chambolle04=False, clip=False,
           clip_alpha=4.0):
    """GAP-TV (Eq. (21)-(22), Algorithm 1). Returns (x^(T), theta^(T)).
    warm_dual: each denoiser call starts from the previous call's final dual;
    clip: the ATV-Clip denoiser (step 1/clip_alpha)."""
    Y, C = _d(Y), _d(C)
    B, nx, ny = _dims(C)
    x = np.empty((B, nx, ny))
    th = np.empty((B, nx, ny))
    xi = None if x_init is None else _d(x_init)
    _load().orc_gap_tv(_kind(tv), B, nx, ny, float(lam), int(T), int(N), int(bool(accel)), int(bool(warm_dual)),
                       _variant(chambolle04, clip, tv), float(clip_alpha), _p(Y), _p(C), _p(xi), _p(x), _p(th))
    return x, th


def admm_tv(Y, C, lam, rho, T, N, tv="atv", accel=True, x_init=None, warm_dual=False, chambolle04=False,
            clip=False, clip_alpha=4.0):
    """ADMM-TV (Eq. (24)-(26)). Returns (x^(T), theta^(T))."""
    Y, C = _d(Y), _d(C)
    B, nx, ny = _dims(C)
    x = np.empty((B, nx, ny))
    th = np.empty((B, nx, ny))
    xi = None if x_init is None else _d(x_init)
    _load().orc_admm_tv(_kind(tv), B, nx, ny, float(lam), float(rho), int(T), int(N), int(bool(accel)),
                        int(bool(warm_dual)), _variant(chambolle04, clip, tv), float(clip_alpha), _p(Y), _p(C),
                        _p(xi), _p(x), _p(th))
    return x, th


def clip_denoise(x, lam, n_iter, alpha=4.0, w_init=None, return_dual=False):
    """ATV-Clip (Sec. 2.3, Algorithm 1): per-direction iterative clipping at
    threshold 2 lam, step 1/alpha."""
    x = _d(x)
    B, nx, ny = _dims(x)
    th = np.empty_like(x)
    wi = None if w_init is None else _d(w_init)
    wh, wv = np.empty_like(x), np.empty_like(x)
    _load().orc_clip_denoise(B, nx, ny, float(lam), float(alpha), int(n_iter), _p(x), _p(wi), _p(th), _p(wh),
                             _p(wv))
    if return_dual:
        return th, np.stack([wh, wv])
    return th


def lipschitz(C):
    """L(f) = max_ij sum_k C_kij^2 (largest eigenvalue of Phi^T Phi)."""
    C = _d(C)
    B, nx, ny = _dims(C)
    return _load().orc_lipschitz(B, nx, ny, _p(C))


def twist_default_ab(xi1=0.1, xim=1.0):
    """TwIST's alpha, beta from the spectrum bounds [xi1, xim] of the scaled
    Phi^T Phi: rho = (1 - sqrt(xi1/xim)) / (1 + sqrt(xi1/xim)),
    alpha = 1 + rho^2, beta = 2 alpha / (xi1 + xim). Phi^T Phi is singular in
    SCI (rank nx*ny of B*nx*ny), so xi1 is a chosen bound, 0.1 by default."""
    k = math.sqrt(xi1 / xim)
    rho = (1.0 - k) / (1.0 + k)
    alpha = 1.0 + rho * rho
    return alpha, 2.0 * alpha / (xi1 + xim)


def fista_tv(Y, C, lam, T, N, tv="atv", accel=True, x_init=None, warm_dual=False):
    """FISTA with the TV prox (Sec. 2.2). Returns (x^(T), theta^(T+1)).
    warm_dual: each prox call starts from the previous call's final dual."""
    Y, C = _d(Y), _d(C)
    B, nx, ny = _dims(C)
    x = np.empty((B, nx, ny))
    th = np.empty((B, nx, ny))
    xi = None if x_init is None else _d(x_init)
    rc = _load().orc_fista_tv(_kind(tv), B, nx, ny, float(lam), int(T), int(N), int(bool(accel)),
                              int(bool(warm_dual)), _p(Y), _p(C), _p(xi), _p(x), _p(th))
    if rc != 0:
        raise ValueError("FISTA needs a nonzero mask (L(f) > 0)")
    return x, th


def twist_tv(Y, C, lam, T, N, tv="atv", alpha=None, beta=None, accel=True, x_init=None, warm_dual=False):
    """TwIST with the TV denoiser (Sec. 2.2). Returns (x^(T), theta^(T-1)).
    warm_dual: each denoiser call starts from the previous call's final dual."""
    if alpha is None or beta is None:
        alpha, beta = twist_default_ab()
    Y, C = _d(Y), _d(C)
    B, nx, ny = _dims(C)
    x = np.empty((B, nx, ny))
    th = np.empty((B, nx, ny))
    xi = None if x_init is None else _d(x_init)
    rc = _load().orc_twist_tv(_kind(tv), B, nx, ny, float(lam), float(alpha), float(beta), int(T), int(N),
                              int(bool(accel)), int(bool(warm_dual)), _p(Y), _p(C), _p(xi), _p(x), _p(th))
    if rc != 0:
        raise ValueError("TwIST needs a nonzero mask (L(f) > 0)")
    return x, th


def psnr(a, ref, peak=1.0):
    a, ref = _d(a), _d(ref)
    return _load().orc_psnr(a.size, _p(a), _p(ref), float(peak))


def residual_sq(C, X, Y):
    C, X, Y = _d(C), _d(X), _d(Y)
    B, nx, ny = _dims(C)
    return _load().orc_residual_sq(B, nx, ny, _p(C), _p(X), _p(Y))


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's element-wise loops (n <= 0: unchanged);
    returns the count in effect. Results do not depend on it."""
    return _load().orc_set_threads(int(n))


def measurement(C, X, G=None):
    """Y = Phi X + G formed in FP64 by the oracle and rounded once to float32."""
    Y = forward(C, X)
    if G is not None:
        Y = Y + _d(G)
    return Y.astype(np.float32)
