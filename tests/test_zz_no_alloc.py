"""GPU: the allocation-free GAP entry point (sci_gap_tv_noalloc) through the
raw C ABI against sci_gap_tv with the same parameters, on two calls in a row
(the second on a smaller problem, so stale scratch contents would show), and
against the FP64 oracle."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import oracle as orc  # noqa: E402
from paper_2005_08028_amd import synth  # noqa: E402


@pytest.fixture(scope="module")
def sc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_08028_amd import scitv
    return scitv


@pytest.fixture(scope="module")
def ctx(sc):
    c = sc.Context(0)
    yield c.handle
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def raw_noalloc(sc, ctx, Y, C, prm, X, Th, X_init=None):
    B, nx, ny = C.shape
    return sc.lib.sci_gap_tv_noalloc(ctx, sc.sci_dims(nx, ny, B), ctypes.byref(prm), ptr(Y), ptr(C), ptr(X),
                                     ptr(Th), ptr(X_init), None)


# (nx, ny, B, tv, n_inner, mask): the second of each pair is smaller than the first
CASES = [
    ((96, 130, 10, "itv2d", 10, "bernoulli"), (40, 66, 8, "itv2d", 10, "bernoulli")),
    ((64, 80, 24, "vtv", 5, "shifted"), (33, 35, 6, "vtv", 5, "bernoulli")),
    ((70, 90, 12, "atv", 7, "graded"), (21, 33, 40, "atv", 3, "bernoulli")),
]


def problem(nx, ny, B, mask, seed):
    pr = synth.make_problem(nx, ny, B, seed=seed, sigma=0.01, radius=(3.0, 15.0),
                            mask="shifted" if mask == "shifted" else "bernoulli")
    C = pr.masks
    if mask == "graded":
        C = (C * np.random.default_rng(seed).uniform(0.2, 1.0, size=C.shape)).astype(np.float32)
    return pr, C, orc.measurement(C, pr.truth, pr.noise)


@pytest.mark.parametrize("pair", CASES, ids=["itv2d", "vtv", "atv_graded_then_b40"])
def test_noalloc_matches_gap_twice(sc, ctx, pair):
    for k, (nx, ny, B, tv, n, mask) in enumerate(pair):
        print(f"noalloc case {tv} {nx}x{ny}x{B} n_inner={n} mask={mask} call {k + 1}", flush=True)
        pr, C, Y = problem(nx, ny, B, mask, seed=nx + ny + B)
        Yd, Cd = dev(Y), dev(C)
        prm = sc.solver_params(outer_iters=6, tv=tv, lam=0.1, n_inner=n, tile_passes=1)
        X = torch.full(C.shape, np.nan, device="cuda")
        Th = torch.full(C.shape, np.nan, device="cuda")
        assert raw_noalloc(sc, ctx, Yd, Cd, prm, X, Th) == sc.SCI_OK, sc.lib.sci_last_error(ctx)
        Th_ref = torch.empty_like(Th)
        X_ref, _ = sc.sci_gap_tv(ctx, Yd, Cd, prm, Theta_out=Th_ref)
        np.testing.assert_array_equal(host(X), host(X_ref))
        np.testing.assert_array_equal(host(Th), host(Th_ref))
        xr, _ = orc.gap_tv(Y, C, float(np.float32(0.1)), 6, n, tv=tv)
        e = np.linalg.norm(host(X) - xr) / np.linalg.norm(xr)
        print(f"  bit-equal to sci_gap_tv; rel-L2 vs oracle {e:.2e}", flush=True)
        assert e <= 1e-4


def test_noalloc_rejects_before_launch(sc, ctx):
    pr, C, Y = problem(16, 20, 4, "bernoulli", seed=5)
    Yd, Cd = dev(Y), dev(C)
    X = torch.empty(C.shape, device="cuda")
    Th = torch.empty(C.shape, device="cuda")
    prm = sc.solver_params(outer_iters=2, tv="atv", lam=0.1, n_inner=5)
    assert raw_noalloc(sc, ctx, Yd, Cd, prm, X, None) == sc.SCI_ERR_INVALID_ARG  # Theta_out required
    big = sc.solver_params(outer_iters=2, tv="atv", lam=0.1, n_inner=5)
    # more pixels than the fixed scratch holds: rejected by the size check, nothing is launched
    st = sc.lib.sci_gap_tv_noalloc(ctx, sc.sci_dims(2049, 2048, 1), ctypes.byref(big), ptr(Yd), ptr(Cd), ptr(X),
                                   ptr(Th), None, None)
    assert st == sc.SCI_ERR_INVALID_ARG and b"4194304" in sc.lib.sci_last_error(ctx)
    for bad in (sc.solver_params(outer_iters=2, tv="atv", lam=0.1, n_inner=11),
                sc.solver_params(outer_iters=2, tv="atv", lam=0.1, n_inner=5, warm_dual=True),
                sc.solver_params(outer_iters=2, tv="atv", lam=0.1, n_inner=5, use_graph=True)):
        assert raw_noalloc(sc, ctx, Yd, Cd, bad, X, Th) == sc.SCI_ERR_UNSUPPORTED
    # the context still works, and the entry point with it
    assert raw_noalloc(sc, ctx, Yd, Cd, prm, X, Th) == sc.SCI_OK
    torch.cuda.synchronize()
