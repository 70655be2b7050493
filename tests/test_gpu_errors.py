"""Argument validation through the raw C ABI on a real context: every call
below is rejected before any kernel is launched, with the documented status
code and a message, and the context keeps working afterwards."""
import ctypes
import math

import numpy as np
import pytest

try:
    import torch
except ImportError:  # pragma: no cover
    torch = None

from oracle import oracle as orc  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sc():
    if torch is None or not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_08028_amd import scitv
    return scitv


@pytest.fixture(scope="module")
def ctx(sc):
    c = sc.Context(0)
    yield c.handle
    c.close()


def ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def stream(sc):
    return sc._stream(None)


@pytest.fixture()
def bufs():
    B, nx, ny = 3, 9, 14
    C = torch.rand((B, nx, ny), device="cuda").round()
    X = torch.rand((B, nx, ny), device="cuda")
    Y = torch.rand((nx, ny), device="cuda")
    out = torch.empty((B, nx, ny), device="cuda")
    return B, nx, ny, C, X, Y, out


def test_forward_adjoint_validation(sc, ctx, bufs):
    B, nx, ny, C, X, Y, out = bufs
    D = sc.sci_dims
    cases = [
        (sc.lib.sci_forward(ctx, D(0, ny, B), ptr(C), ptr(X), ptr(Y), stream(sc)), sc.SCI_ERR_INVALID_ARG),
        (sc.lib.sci_forward(ctx, D(nx, ny, B), None, ptr(X), ptr(Y), stream(sc)), sc.SCI_ERR_INVALID_ARG),
        (sc.lib.sci_forward(ctx, D(1 << 12, 1 << 12, 128), ptr(C), ptr(X), ptr(Y), stream(sc)),
         sc.SCI_ERR_INVALID_ARG),  # B nx ny >= 2^31
        (sc.lib.sci_forward(ctx, D(nx, ny, B), ptr(C), ptr(X), ptr(X), stream(sc)), sc.SCI_ERR_ALIAS),
        (sc.lib.sci_adjoint(ctx, D(nx, ny, B), ptr(C), ptr(Y), ptr(C), stream(sc)), sc.SCI_ERR_ALIAS),
    ]
    for st, want in cases:
        assert st == want
        assert sc.lib.sci_last_error(ctx).decode()


def gap_call(sc, ctx, d, prm, Y, C, out, theta=None):
    return sc.lib.sci_gap_tv(ctx, d, ctypes.byref(prm), ptr(Y), ptr(C), ptr(out),
                             ptr(theta) if theta is not None else None, None, stream(sc))


def test_solver_validation(sc, ctx, bufs):
    B, nx, ny, C, X, Y, out = bufs
    D = sc.sci_dims
    d = D(nx, ny, B)
    good = dict(outer_iters=2, tv="itv2d", lam=0.1, n_inner=3)

    def prm(**kw):
        p = dict(good)
        p.update(kw)
        return sc.solver_params(**p)

    cases = [
        (dict(lam=-1.0), sc.SCI_ERR_INVALID_ARG),
        (dict(lam=math.nan), sc.SCI_ERR_INVALID_ARG),
        (dict(n_inner=-1), sc.SCI_ERR_INVALID_ARG),
        (dict(tv=7), sc.SCI_ERR_INVALID_ARG),
        (dict(dual_dtype=5), sc.SCI_ERR_INVALID_ARG),
        (dict(schedule=9), sc.SCI_ERR_INVALID_ARG),
        (dict(tile_shape=99), sc.SCI_ERR_INVALID_ARG),
        (dict(rho=-0.5), sc.SCI_ERR_INVALID_ARG),
        (dict(outer_iters=-3), sc.SCI_ERR_INVALID_ARG),
        (dict(chambolle04=True, dual_dtype="bf16", schedule="fused"), sc.SCI_ERR_UNSUPPORTED),
        (dict(clip=True, tv="itv2d"), sc.SCI_ERR_INVALID_ARG),  # ATV-Clip is defined for ATV only
    ]
    for kw, want in cases:
        st = gap_call(sc, ctx, d, prm(**kw), Y, C, out)
        msg = sc.lib.sci_last_error(ctx).decode()
        assert st == want, (kw, st, msg)
        assert msg, kw
    # VTV couples all frames of a pixel: at most 48, and at most 32 on the fused schedule
    for B2, kw in ((49, dict()), (33, dict(schedule="fused"))):
        C2 = torch.ones((B2, 4, 5), device="cuda")
        Y2 = torch.ones((4, 5), device="cuda")
        o2 = torch.empty((B2, 4, 5), device="cuda")
        assert gap_call(sc, ctx, D(4, 5, B2), prm(tv="vtv", **kw), Y2, C2, o2) == sc.SCI_ERR_UNSUPPORTED
    # outputs overlapping inputs
    assert gap_call(sc, ctx, d, prm(), Y, C, C) == sc.SCI_ERR_ALIAS
    assert gap_call(sc, ctx, d, prm(), Y, C, out, theta=out) != sc.SCI_OK
    # null inputs
    st = sc.lib.sci_gap_tv(ctx, d, ctypes.byref(prm()), None, ptr(C), ptr(out), None, None, stream(sc))
    assert st == sc.SCI_ERR_INVALID_ARG


def test_denoise_validation(sc, ctx, bufs):
    B, nx, ny, C, X, Y, out = bufs
    d = sc.sci_dims(nx, ny, B)
    f = sc.lib.sci_tv_denoise

    def call(p, x=X, th=out):
        return f(ctx, d, ctypes.byref(p), ptr(x), ptr(th), None, None, None, None, stream(sc))

    assert call(sc.tv_params(tv="atv", gap_tol=1e-4, n_inner_max=0)) == sc.SCI_ERR_INVALID_ARG
    assert call(sc.tv_params(tv="atv", gap_tol=math.inf, n_inner_max=10)) == sc.SCI_ERR_INVALID_ARG
    assert call(sc.tv_params(tv="atv"), th=X) == sc.SCI_ERR_ALIAS
    st = f(ctx, d, ctypes.byref(sc.tv_params(tv="atv")), ptr(X), None, None, None, None, None, stream(sc))
    assert st == sc.SCI_ERR_INVALID_ARG


def test_context_still_works_after_errors(sc, ctx, bufs):
    """A valid call after the rejected ones returns the right result."""
    B, nx, ny, C, X, Y, out = bufs
    assert sc.lib.sci_forward(ctx, sc.sci_dims(0, 0, 0), None, None, None, stream(sc)) == sc.SCI_ERR_INVALID_ARG
    Yg = sc.sci_forward(ctx, C, X)
    ref = orc.forward(C.cpu().numpy(), X.cpu().numpy())
    np.testing.assert_allclose(Yg.cpu().numpy(), ref, rtol=1e-6, atol=1e-6)
    for code in (sc.SCI_OK, sc.SCI_NOT_CONVERGED, sc.SCI_ERR_INVALID_ARG, sc.SCI_ERR_ALIAS, sc.SCI_ERR_NOMEM,
                 sc.SCI_ERR_HIP, sc.SCI_ERR_UNSUPPORTED):
        assert sc.lib.sci_status_string(code)
