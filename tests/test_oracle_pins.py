"""Pins for the FP64 oracle, each independent of the oracle's own code.

Every check below compares the oracle with something fixed by the paper or by
mathematics: the dense matrices that Eq. (2) and Eq. (7) define, closed-form
TV values and prox solutions, hand-derived worked examples, an independent
bound-constrained solve of the denoising dual with scipy, optimality
certificates computed with dense matrices, fixed points and normal equations.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.optimize

from oracle import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fgp_worked_examples.json")


def rng(seed=0):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------------------
# Dense reference matrices, written straight from the definitions.
# ---------------------------------------------------------------------------

def dense_phi(C):
    """Phi = [D_1, ..., D_B], D_k = diag(vec(C_k)) (Eq. (2), (5)); vec stacks columns."""
    B = C.shape[0]
    return np.hstack([np.diag(C[k].ravel(order="F")) for k in range(B)])


def vec_video(X):
    return np.concatenate([X[k].ravel(order="F") for k in range(X.shape[0])])


def unvec_video(x, B, nx, ny):
    n = nx * ny
    return np.stack([x[k * n:(k + 1) * n].reshape((nx, ny), order="F") for k in range(B)])


def diff_matrix(n):
    """(n-1) x n forward-difference matrix: row r = e_{r+1} - e_r (Eq. (7) sizes)."""
    D = np.zeros((max(n - 1, 0), n))
    for r in range(n - 1):
        D[r, r] = -1.0
        D[r, r + 1] = 1.0
    return D


def dense_grad(X):
    """D_h x_k = X_k D_h^T, D_v x_k = D_v X_k (Eq. (7)), zero-padded to full size."""
    B, nx, ny = X.shape
    Dh, Dv = diff_matrix(ny), diff_matrix(nx)
    gh = np.zeros_like(X)
    gv = np.zeros_like(X)
    for k in range(B):
        gh[k, :, :ny - 1] = X[k] @ Dh.T
        gv[k, :nx - 1, :] = Dv @ X[k]
    return np.stack([gh, gv])


def dense_grad_adj(p):
    _, B, nx, ny = p.shape
    Dh, Dv = diff_matrix(ny), diff_matrix(nx)
    out = np.zeros((B, nx, ny))
    for k in range(B):
        out[k] += p[0, k, :, :ny - 1] @ Dh
        out[k] += Dv.T @ p[1, k, :nx - 1, :]
    return out


def dense_tv(theta, tv):
    g = dense_grad(theta)
    if tv == "atv":
        return np.abs(g).sum()
    if tv == "itv2d":
        return np.sqrt(g[0] ** 2 + g[1] ** 2).sum()
    return np.sqrt((g[0] ** 2 + g[1] ** 2).sum(axis=0)).sum()


def dual_norm_max(p, tv):
    if tv == "atv":
        return np.abs(p).max()
    if tv == "itv2d":
        return np.sqrt(p[0] ** 2 + p[1] ** 2).max()
    return np.sqrt((p[0] ** 2 + p[1] ** 2).sum(axis=0)).max()


def certificate_gap(x, p, lam, tv):
    """Primal minus dual objective with dense operators: an optimality
    certificate of theta = x - lam D^T p that does not use the oracle's code."""
    th = x - lam * dense_grad_adj(p)
    primal = 0.5 * ((th - x) ** 2).sum() + lam * dense_tv(th, tv)
    dual = 0.5 * (x ** 2).sum() - 0.5 * ((x - lam * dense_grad_adj(p)) ** 2).sum()
    return primal - dual, primal


# ---------------------------------------------------------------------------
# Sensing operator Phi, Phi^T (Eq. (2)-(5)).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("B,nx,ny", [(1, 3, 4), (3, 5, 2), (4, 6, 7)])
def test_forward_adjoint_match_dense_phi(B, nx, ny):
    r = rng(1)
    C = r.uniform(size=(B, nx, ny))
    X = r.normal(size=(B, nx, ny))
    Yv = r.normal(size=(nx, ny))
    Phi = dense_phi(C)
    y = Phi @ vec_video(X)
    np.testing.assert_allclose(orc.forward(C, X).ravel(order="F"), y, rtol=1e-13, atol=1e-13)
    xa = Phi.T @ Yv.ravel(order="F")
    np.testing.assert_allclose(vec_video(orc.adjoint(C, Yv)), xa, rtol=1e-13, atol=1e-13)
    # adjoint identity <Phi x, y> = <x, Phi^T y>
    lhs = (orc.forward(C, X) * Yv).sum()
    rhs = (X * orc.adjoint(C, Yv)).sum()
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_forward_special_masks():
    r = rng(2)
    X = r.normal(size=(5, 4, 6))
    np.testing.assert_allclose(orc.forward(np.ones_like(X), X), X.sum(axis=0), rtol=1e-14)
    C = np.zeros_like(X)
    C[3] = 1.0
    np.testing.assert_array_equal(orc.forward(C, X), X[3])


def test_weights_diag_phiphit():
    r = rng(3)
    C = (r.uniform(size=(4, 5, 6)) < 0.5).astype(float)
    C[:, 0, 0] = 0.0  # a pixel no frame sees
    Phi = dense_phi(C)
    S = np.diag(Phi @ Phi.T).reshape((5, 6), order="F")
    W = orc.weights(C)
    expect = np.where(S > 0, 1.0 / np.where(S > 0, S, 1.0), 0.0)
    np.testing.assert_allclose(W, expect, rtol=1e-15)
    assert W[0, 0] == 0.0
    np.testing.assert_allclose(orc.weights(C, 0.5), 1.0 / (S + 0.5), rtol=1e-15)


# ---------------------------------------------------------------------------
# Finite differences (Eq. (7)).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("B,nx,ny", [(1, 1, 1), (1, 1, 5), (2, 4, 1), (2, 5, 7), (3, 8, 3)])
def test_grad_matches_dense_difference_matrices(B, nx, ny):
    r = rng(4)
    X = r.normal(size=(B, nx, ny))
    p = r.normal(size=(2, B, nx, ny))
    np.testing.assert_allclose(orc.grad(X), dense_grad(X), rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(orc.grad_adj(p), dense_grad_adj(p), rtol=1e-13, atol=1e-13)
    lhs = (orc.grad(X) * p).sum()
    rhs = (X * orc.grad_adj(p)).sum()
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_grad_of_constant_is_zero():
    assert np.abs(orc.grad(np.full((3, 6, 5), 2.5))).max() == 0.0


def test_dtd_norm_below_eight():
    """||D^T D|| approaches 8 from below (the 1/(8 lambda) step of Algorithm 1)."""
    r = rng(5)
    v = r.normal(size=(1, 48, 48))
    for _ in range(600):
        v = orc.grad_adj(orc.grad(v))
        nrm = np.sqrt((v ** 2).sum())
        v /= nrm
    assert 7.9 < nrm < 8.0


# ---------------------------------------------------------------------------
# TV values (Eq. (8)-(10), per-pixel reading).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_tv_closed_forms(tv):
    nx, ny, B, h, m = 7, 9, 4, 0.35, 4
    assert orc.tv_value(np.full((B, nx, ny), 0.3), tv) == 0.0
    step = np.zeros((B, nx, ny))
    step[:, :, m:] = h  # identical frames, a jump of height h across every row
    expect = {"atv": B * nx * h, "itv2d": B * nx * h, "vtv": math.sqrt(B) * nx * h}[tv]
    assert abs(orc.tv_value(step, tv) - expect) < 1e-12
    X = rng(6).normal(size=(B, nx, ny))
    assert abs(orc.tv_value(X, tv) - dense_tv(X, tv)) < 1e-10 * dense_tv(X, tv)


@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_project_dual_is_ball_projection(tv):
    r = rng(7)
    q = r.normal(size=(2, 3, 4, 5)) * 2.0
    p = orc.project_dual(q, tv)
    assert dual_norm_max(p, tv) <= 1.0 + 1e-15
    # the projection onto a convex set is firmly non-expansive and idempotent
    np.testing.assert_allclose(orc.project_dual(p, tv), p, rtol=0, atol=1e-15)
    if tv == "atv":
        np.testing.assert_allclose(p, np.clip(q, -1, 1), rtol=0, atol=1e-15)
    else:
        axes = (0,) if tv == "itv2d" else (0, 1)
        nq = np.sqrt((q ** 2).sum(axis=axes, keepdims=True))
        np.testing.assert_allclose(p, q / np.maximum(1.0, nq), rtol=1e-15)


def test_fgp_beta_recursion():
    b = orc.fgp_beta(4)
    nu1 = (1 + math.sqrt(5)) / 2
    nu2 = (1 + math.sqrt(1 + 4 * nu1 * nu1)) / 2
    assert b[0] == 0.0
    assert abs(b[1] - (nu1 - 1) / nu2) < 1e-15


# ---------------------------------------------------------------------------
# TV denoiser (Algorithm 1 FGP / Cham boxes, Eq. (27)-(32)).
# ---------------------------------------------------------------------------

def test_golden_worked_example_2x2():
    g = json.load(open(GOLDEN))["cases"][0]
    x = np.array(g["x"], dtype=float)
    for n in (1, 2, 7):
        th, p = orc.tv_denoise(x, g["lam"], n, g["tv"], return_dual=True)
        np.testing.assert_allclose(th, np.array(g["theta"]), rtol=0, atol=1e-15)
        np.testing.assert_allclose(p[0], np.array(g["p_h"]), rtol=0, atol=1e-15)
        np.testing.assert_allclose(p[1], np.array(g["p_v"]), rtol=0, atol=1e-15)
        gap, _ = orc.dual_gap(x, p, g["lam"], g["tv"])
        assert abs(gap - g["gap"]) < 1e-15


@pytest.mark.parametrize("case", [1, 2])
def test_golden_step_closed_form(case):
    g = json.load(open(GOLDEN))["cases"][case]
    B = g.get("B", 1)
    nx = 3
    x = np.full((B, nx, g["n"]), g["a"])
    x[:, :, g["m"]:] = g["b"]
    tvs = g["tv"] if isinstance(g["tv"], list) else [g["tv"]]
    for tv in tvs:
        th = orc.tv_denoise(x, g["lam"], 3000, tv)
        np.testing.assert_allclose(th[:, :, :g["m"]], g["left"], rtol=0, atol=1e-9)
        np.testing.assert_allclose(th[:, :, g["m"]:], g["right"], rtol=0, atol=1e-9)


@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_denoiser_identities(tv):
    r = rng(8)
    B, nx, ny = 3, 9, 11
    x = r.uniform(size=(B, nx, ny))
    lam = 0.07
    # lambda = 0 and N = 0 return the input
    np.testing.assert_array_equal(orc.tv_denoise(x, 0.0, 5, tv), x)
    np.testing.assert_array_equal(orc.tv_denoise(x, lam, 0, tv), x)
    # constant input is a fixed point
    c = np.full((B, nx, ny), 0.4)
    np.testing.assert_allclose(orc.tv_denoise(c, lam, 6, tv), c, rtol=0, atol=1e-15)
    base = orc.tv_denoise(x, lam, 6, tv)
    # per-frame constant shifts pass through (D kills constants)
    shift = np.array([0.5, -1.25, 3.0])[:, None, None]
    np.testing.assert_allclose(orc.tv_denoise(x + shift, lam, 6, tv), base + shift, rtol=0, atol=1e-12)
    # positive homogeneity: TVD_{a lam}(a x) = a TVD_lam(x)
    a = 2.5
    np.testing.assert_allclose(orc.tv_denoise(a * x, a * lam, 6, tv), a * base, rtol=0, atol=1e-12)


def test_vtv_single_frame_equals_itv2d():
    x = rng(9).uniform(size=(1, 10, 8))
    np.testing.assert_allclose(orc.tv_denoise(x, 0.1, 9, "vtv"), orc.tv_denoise(x, 0.1, 9, "itv2d"),
                               rtol=0, atol=0)


def test_identical_rows_atv_equals_itv2d():
    row = rng(10).uniform(size=(2, 1, 13))
    x = np.repeat(row, 6, axis=1)
    np.testing.assert_allclose(orc.tv_denoise(x, 0.1, 9, "atv"), orc.tv_denoise(x, 0.1, 9, "itv2d"),
                               rtol=0, atol=1e-15)


def scipy_atv_prox(x, lam):
    """Independent ATV prox: minimise 1/2 ||x - lam D^T p||^2 over the box
    |p| <= 1 (entries without a difference fixed to 0) with L-BFGS-B on the
    dense difference matrices."""
    B, nx, ny = x.shape
    mask = np.zeros((2, B, nx, ny), bool)
    mask[0, :, :, :ny - 1] = True
    mask[1, :, :nx - 1, :] = True
    idx = np.flatnonzero(mask)

    def unpack(z):
        p = np.zeros(mask.size)
        p[idx] = z
        return p.reshape(mask.shape)

    def f(z):
        p = unpack(z)
        res = x - lam * dense_grad_adj(p)
        g = -lam * dense_grad(res)
        return 0.5 * (res ** 2).sum(), g.ravel()[idx]

    z0 = np.zeros(idx.size)
    out = scipy.optimize.minimize(f, z0, jac=True, method="L-BFGS-B", bounds=[(-1, 1)] * idx.size,
                                  options=dict(maxiter=20000, ftol=1e-15, gtol=1e-12))
    return x - lam * dense_grad_adj(unpack(out.x))


def test_atv_fgp_converges_to_independent_prox():
    x = rng(11).uniform(size=(2, 6, 7))
    lam = 0.08
    ref = scipy_atv_prox(x, lam)
    th = orc.tv_denoise(x, lam, 4000, "atv")
    np.testing.assert_allclose(th, ref, rtol=0, atol=2e-6)


@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_denoiser_gap_certificate_and_convergence(tv):
    """The oracle's dual is feasible and its dense-matrix duality gap, which
    bounds the distance to the unique prox, goes to zero; the oracle's own
    gap routine agrees with the dense certificate."""
    x = rng(12).uniform(size=(4, 16, 16))
    lam = 0.1
    prev = np.inf
    for n in (5, 20, 80, 400):
        th, p = orc.tv_denoise(x, lam, n, tv, return_dual=True)
        assert dual_norm_max(p, tv) <= 1.0 + 1e-12
        cg, prim = certificate_gap(x, p, lam, tv)
        og, oprim = orc.dual_gap(x, p, lam, tv)
        assert cg >= -1e-12
        assert abs(cg - og) <= 1e-9 * max(1.0, prim)
        assert abs(prim - oprim) <= 1e-10 * prim
        np.testing.assert_allclose(th, x - lam * dense_grad_adj(p), rtol=0, atol=1e-13)
        assert cg <= prev * 1.05 + 1e-14
        prev = cg
    assert prev / prim < 1e-6
    # the long-run Chambolle projected gradient reaches the same prox
    th_pg = orc.tv_denoise(x, lam, 20000, tv, accel=False)
    th_fgp = orc.tv_denoise(x, lam, 3000, tv)
    assert np.sqrt(((th_pg - th_fgp) ** 2).sum() / (th_fgp ** 2).sum()) < 1e-5


@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_denoiser_variants_reach_same_prox(tv):
    """Chambolle-2004 denominator and the literal FGP output converge to the same prox."""
    x = rng(13).uniform(size=(2, 8, 9))
    lam = 0.1
    ref = orc.tv_denoise(x, lam, 3000, tv)
    lit = orc.tv_denoise(x, lam, 3000, tv, literal_out=True)
    ch = orc.tv_denoise(x, lam, 20000, tv, accel=False, chambolle04=True)
    assert np.abs(lit - ref).max() < 1e-6
    assert np.abs(ch - ref).max() < 1e-4


def test_large_lambda_gives_frame_means():
    x = rng(14).uniform(size=(3, 6, 6))
    th = orc.tv_denoise(x, 50.0, 3000, "itv2d")
    np.testing.assert_allclose(th, np.broadcast_to(x.mean(axis=(1, 2), keepdims=True), x.shape),
                               rtol=0, atol=1e-6)


def test_warm_start_from_converged_dual_is_fixed():
    x = rng(15).uniform(size=(2, 7, 7))
    th, p = orc.tv_denoise(x, 0.1, 3000, "vtv", return_dual=True)
    th2 = orc.tv_denoise(x, 0.1, 1, "vtv", p_init=p)
    assert np.abs(th2 - th).max() < 1e-7


# ---------------------------------------------------------------------------
# GAP (Eq. (21)-(22)) and ADMM (Eq. (24)-(26)).
# ---------------------------------------------------------------------------

def small_problem(seed=16, B=3, nx=5, ny=6, p=0.5):
    r = rng(seed)
    C = (r.uniform(size=(B, nx, ny)) < p).astype(float)
    X = r.uniform(size=(B, nx, ny))
    return C, X, orc.forward(C, X)


def test_gap_projection_matches_dense_pseudo_inverse():
    C, X, Y = small_problem()
    C[:, 1, 2] = 0.0  # pixel with S = 0
    Y = orc.forward(C, X)
    th0 = rng(17).normal(size=X.shape)
    x, th = orc.gap_tv(Y, C, 0.1, 1, 0, x_init=th0)  # N = 0: denoiser is the identity
    Phi = dense_phi(C)
    y = Y.ravel(order="F")
    ref = vec_video(th0) + Phi.T @ np.linalg.pinv(Phi @ Phi.T) @ (y - Phi @ vec_video(th0))
    np.testing.assert_allclose(vec_video(x), ref, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(th, x)


def test_gap_iterates_satisfy_measurement():
    C, X, Y = small_problem(18, B=4, nx=12, ny=10)
    S = (C ** 2).sum(axis=0)
    for T in (1, 3):
        x, _ = orc.gap_tv(Y, C, 0.1, T, 5, tv="itv2d")
        fx = orc.forward(C, x)
        np.testing.assert_allclose(fx[S > 0], Y[S > 0], rtol=0, atol=1e-12)


def test_gap_single_frame_full_mask_returns_measurement():
    Y = rng(19).uniform(size=(6, 7))
    C = np.ones((1, 6, 7))
    x, _ = orc.gap_tv(Y, C, 0.2, 2, 4, tv="atv")
    np.testing.assert_allclose(x[0], Y, rtol=0, atol=1e-14)


@pytest.mark.parametrize("solver", ["gap", "admm"])
@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_constant_frames_are_fixed_points(solver, tv):
    B, nx, ny = 4, 9, 8
    truth = np.broadcast_to(np.array([0.2, 0.5, 0.9, 0.1])[:, None, None], (B, nx, ny)).copy()
    C = (rng(20).uniform(size=(B, nx, ny)) < 0.5).astype(float)
    Y = orc.forward(C, truth)
    if solver == "gap":
        x, th = orc.gap_tv(Y, C, 0.1, 5, 5, tv=tv, x_init=truth)
    else:
        x, th = orc.admm_tv(Y, C, 0.1, 0.01, 5, 5, tv=tv, x_init=truth)
    np.testing.assert_allclose(x, truth, rtol=0, atol=1e-13)
    np.testing.assert_allclose(th, truth, rtol=0, atol=1e-13)


def test_admm_x_update_solves_normal_equations():
    C, X, Y = small_problem(21)
    rho = 0.3
    v = rng(22).normal(size=X.shape)
    x, th = orc.admm_tv(Y, C, 0.1, rho, 1, 0, x_init=v)  # u0 = 0 -> v = theta0
    Phi = dense_phi(C)
    A = Phi.T @ Phi + rho * np.eye(Phi.shape[1])
    ref = np.linalg.solve(A, Phi.T @ Y.ravel(order="F") + rho * vec_video(v))
    np.testing.assert_allclose(vec_video(x), ref, rtol=0, atol=1e-12)


def test_admm_rho_zero_first_step_is_gap():
    C, X, Y = small_problem(23, B=4, nx=10, ny=9)
    xg, tg = orc.gap_tv(Y, C, 0.1, 1, 6, tv="vtv")
    xa, ta = orc.admm_tv(Y, C, 0.1, 0.0, 1, 6, tv="vtv")
    np.testing.assert_array_equal(xg, xa)
    np.testing.assert_array_equal(tg, ta)


def test_gap_improves_reconstruction():
    """Sanity of the whole loop on a small scene: PSNR rises well above the
    back-projection's."""
    from paper_2005_08028_amd import synth
    pr = synth.make_problem(64, 64, 8, seed=24)
    Y = orc.measurement(pr.masks, pr.truth)
    x0 = orc.adjoint(pr.masks, Y) * orc.weights(pr.masks)[None] * 8 / 8
    x, _ = orc.gap_tv(Y, pr.masks, 0.1, 30, 5, tv="atv")
    assert orc.psnr(x, pr.truth) > orc.psnr(x0, pr.truth) + 8.0


# ---------------------------------------------------------------------------
# Metrics.
# ---------------------------------------------------------------------------

def test_psnr_closed_form():
    ref = rng(25).uniform(size=(3, 4, 5))
    assert abs(orc.psnr(ref + 0.01, ref) - 40.0) < 1e-9
    assert abs(orc.psnr(ref - 0.1, ref, peak=2.0) - 20 * math.log10(20.0)) < 1e-9


def test_residual_sq():
    C, X, Y = small_problem(26)
    assert orc.residual_sq(C, X, Y) < 1e-28
    assert abs(orc.residual_sq(C, X, Y + 0.5) - 0.25 * Y.size) < 1e-12


def test_golden_three_iterations_pin_momentum():
    g = json.load(open(GOLDEN))["cases"][3]
    x = np.array(g["x"], dtype=float)
    for n, ref in g["by_n"].items():
        th, p = orc.tv_denoise(x, g["lam"], int(n), g["tv"], return_dual=True)
        np.testing.assert_allclose(th[0, 0], ref["theta"], rtol=0, atol=1e-15)
        np.testing.assert_allclose(p[0, 0, 0], ref["p_h"], rtol=0, atol=1e-15)
    th = orc.tv_denoise(x, g["lam"], 500, g["tv"])
    np.testing.assert_allclose(th[0, 0], g["converged_theta"], rtol=0, atol=1e-12)


@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_fgp_and_pg_rate_bounds(tv):
    """Beck-Teboulle bounds on the dual objective h(p) = 1/2 ||x - lam D^T p||^2
    (gradient Lipschitz constant L = 8 lam^2, step 1/L): FGP
    h(p_N) - h* <= 2 L ||p0 - p*||^2 / (N+1)^2, projected gradient
    h(p_N) - h* <= L ||p0 - p*||^2 / (2N), from p0 = 0."""
    x = rng(27).uniform(size=(3, 12, 12))
    lam = 0.1
    L = 8 * lam * lam
    th_star, p_star = orc.tv_denoise(x, lam, 20000, tv, return_dual=True)
    h_star = 0.5 * (th_star ** 2).sum()
    R2 = (p_star ** 2).sum()
    for n in (1, 2, 3, 5, 10, 30, 100):
        th = orc.tv_denoise(x, lam, n, tv)
        assert 0.5 * (th ** 2).sum() - h_star <= 2 * L * R2 / (n + 1) ** 2 + 1e-12
        th = orc.tv_denoise(x, lam, n, tv, accel=False)
        assert 0.5 * (th ** 2).sum() - h_star <= L * R2 / (2 * n) + 1e-12


# ---------------------------------------------------------------------------
# Denoiser and outer-loop variants: Chambolle-2004 denominator, warm dual.
# ---------------------------------------------------------------------------

def kind_norm(z, tv):
    """|z| measured per the TV kind, broadcast to z's shape."""
    if tv == "atv":
        return np.abs(z)
    if tv == "itv2d":
        return np.broadcast_to(np.sqrt(z[0] ** 2 + z[1] ** 2), z.shape)
    return np.broadcast_to(np.sqrt((z[0] ** 2 + z[1] ** 2).sum(axis=0)), z.shape)


@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_chambolle04_first_step_closed_form(tv):
    """One semi-implicit step from p = 0: z = D x, p1 = (z/(8 lam)) / (1 + |z|/(8 lam))
    with |z| per the TV kind, theta = x - lam D^T p1 (dense D)."""
    x = rng(40).uniform(size=(3, 6, 7))
    lam = 0.15
    st = 1.0 / (8 * lam)
    z = dense_grad(x)
    p1 = st * z / (1.0 + st * kind_norm(z, tv))
    th, p = orc.tv_denoise(x, lam, 1, tv, accel=False, chambolle04=True, return_dual=True)
    np.testing.assert_allclose(p, p1, rtol=0, atol=1e-14)
    np.testing.assert_allclose(th, x - lam * dense_grad_adj(p1), rtol=0, atol=1e-14)
    # the step stays inside the dual ball without a projection
    assert dual_norm_max(p, tv) < 1.0


def explicit_gap(Y, C, lam, T, N, tv, warm):
    """GAP written out from the primitives, the dual carried by hand."""
    S = orc.weights(C)
    th = orc.adjoint(C, Y)
    p = None
    for _ in range(T):
        x = th + orc.adjoint(C, (Y - orc.forward(C, th)) * S)
        th, pn = orc.tv_denoise(x, lam, N, tv, p_init=p if warm else None, return_dual=True)
        p = pn
    return x, th


@pytest.mark.parametrize("tv", ["atv", "vtv"])
def test_warm_dual_gap(tv):
    C, X, Y = small_problem(41, B=3, nx=9, ny=8)
    # driver against the loop written out
    xw, tw = orc.gap_tv(Y, C, 0.1, 4, 3, tv=tv, warm_dual=True)
    xe, te = explicit_gap(Y, C, 0.1, 4, 3, tv, warm=True)
    np.testing.assert_allclose(xw, xe, rtol=0, atol=1e-14)
    np.testing.assert_allclose(tw, te, rtol=0, atol=1e-14)
    # one outer iteration has no previous dual: same as the cold start
    np.testing.assert_array_equal(orc.gap_tv(Y, C, 0.1, 1, 3, tv=tv, warm_dual=True)[0],
                                  orc.gap_tv(Y, C, 0.1, 1, 3, tv=tv)[0])
    # few inner iterations: the start matters
    xc, _ = orc.gap_tv(Y, C, 0.1, 4, 3, tv=tv)
    assert np.abs(xc - xw).max() > 1e-6
    # converged inner solves: the prox is unique, so the start does not matter
    xw, _ = orc.gap_tv(Y, C, 0.1, 3, 3000, tv=tv, warm_dual=True)
    xc, _ = orc.gap_tv(Y, C, 0.1, 3, 3000, tv=tv)
    assert np.abs(xc - xw).max() < 1e-7


def test_warm_dual_admm_and_chambolle04_outer():
    C, X, Y = small_problem(42, B=3, nx=7, ny=8)
    xw, _ = orc.admm_tv(Y, C, 0.1, 0.05, 3, 3000, tv="itv2d", warm_dual=True)
    xc, _ = orc.admm_tv(Y, C, 0.1, 0.05, 3, 3000, tv="itv2d")
    assert np.abs(xc - xw).max() < 1e-7
    xw, _ = orc.admm_tv(Y, C, 0.1, 0.05, 3, 4, tv="itv2d", warm_dual=True)
    xc, _ = orc.admm_tv(Y, C, 0.1, 0.05, 3, 4, tv="itv2d")
    assert np.abs(xc - xw).max() > 1e-6
    # the semi-implicit denoiser converges to the same prox inside GAP
    xs, _ = orc.gap_tv(Y, C, 0.1, 2, 3000, tv="itv2d")
    xh, _ = orc.gap_tv(Y, C, 0.1, 2, 20000, tv="itv2d", accel=False, chambolle04=True)
    assert np.abs(xs - xh).max() < 1e-4


def explicit_prox_grad(Y, C, lam, T, N, tv, warm, twist, alpha=None, beta=None):
    """FISTA (twist = False) or TwIST written out from the primitives, the
    prox dual carried by hand when warm."""
    L = orc.lipschitz(C)
    x = orc.adjoint(C, Y)
    th = x.copy()
    xp = None
    tau, p = 1.0, None
    for t in range(T):
        base = x if twist else th
        z = base + orc.adjoint(C, Y - orc.forward(C, base)) / L
        d, pn = orc.tv_denoise(z, lam / L, N, tv, p_init=p if warm else None, return_dual=True)
        p = pn
        if twist:
            th = d
            if t == 0:
                xp, x = x, d
            else:
                xp, x = x, (1.0 - alpha) * xp + (alpha - beta) * x + beta * d
        else:
            xp, x = x, d
            tau1 = (1.0 + math.sqrt(1.0 + 4.0 * tau * tau)) / 2.0
            th = x + (tau - 1.0) / tau1 * (x - xp)
            tau = tau1
    return x, th


@pytest.mark.parametrize("twist", [False, True])
def test_warm_dual_fista_twist(twist):
    """Warm duals in FISTA / TwIST (each prox call starts from the previous
    call's final dual): the drivers equal the loops written out with the
    dual carried by hand; one outer iteration equals the cold start; with few
    inner iterations the start matters, with converged inner solves it does
    not (the prox is unique)."""
    C, X, Y = small_problem(43, B=3, nx=9, ny=8)
    a, b = orc.twist_default_ab()

    def run(T, N, warm):
        if twist:
            return orc.twist_tv(Y, C, 0.1, T, N, tv="itv2d", alpha=a, beta=b, warm_dual=warm)
        return orc.fista_tv(Y, C, 0.1, T, N, tv="itv2d", warm_dual=warm)

    for warm in (False, True):
        xw, tw = run(4, 3, warm)
        xe, te = explicit_prox_grad(Y, C, 0.1, 4, 3, "itv2d", warm, twist, a, b)
        np.testing.assert_allclose(xw, xe, rtol=0, atol=1e-13)
        np.testing.assert_allclose(tw, te, rtol=0, atol=1e-13)
    np.testing.assert_array_equal(run(1, 3, True)[0], run(1, 3, False)[0])
    assert np.abs(run(4, 3, True)[0] - run(4, 3, False)[0]).max() > 1e-6
    assert np.abs(run(3, 3000, True)[0] - run(3, 3000, False)[0]).max() < 1e-7


# ---------------------------------------------------------------------------
# FISTA and TwIST (Sec. 2.2) for 1/2 ||y - Phi x||^2 + lambda TV(x).
# ---------------------------------------------------------------------------

def objective(Y, C, x, lam, tv):
    return 0.5 * orc.residual_sq(C, x, Y) + lam * orc.tv_value(x, tv)


def test_lipschitz_is_largest_eigenvalue():
    C, _, _ = small_problem(50, B=3, nx=4, ny=5)
    Phi = dense_phi(C)
    assert abs(np.linalg.eigvalsh(Phi.T @ Phi).max() - orc.lipschitz(C)) < 1e-12
    C = rng(51).uniform(size=(2, 3, 4))
    Phi = dense_phi(C)
    assert abs(np.linalg.eigvalsh(Phi.T @ Phi).max() - orc.lipschitz(C)) < 1e-12


@pytest.mark.parametrize("tv", ["atv", "itv2d"])
def test_scaled_identity_sensing_reduces_to_one_prox(tv):
    """Phi = c I (one frame, every mask entry c): the objective is
    c^2/2 ||x - y/c||^2 + lambda TV(x), whose minimiser is prox_{lambda/c^2 TV}(y/c).
    The gradient step lands on y/c from any point, so FISTA and TwIST with
    alpha = 1 return that prox at every T >= 1 (checks the 1/L step and the
    lambda/L denoiser weight)."""
    c, lam = 2.0, 0.3
    Y = rng(52).uniform(size=(9, 11))
    C = np.full((1, 9, 11), c)
    ref = orc.tv_denoise(Y[None] / c, lam / c ** 2, 400, tv)
    for T in (1, 2, 5):
        xf, _ = orc.fista_tv(Y, C, lam, T, 400, tv=tv)
        np.testing.assert_allclose(xf, ref, rtol=0, atol=1e-13)
        xt, _ = orc.twist_tv(Y, C, lam, T, 400, tv=tv, alpha=1.0, beta=0.7)
        np.testing.assert_allclose(xt, ref, rtol=0, atol=1e-13)


def test_fista_rate_and_fixed_point():
    """With accurate proximal steps: the Beck-Teboulle bound
    F(x_k) - F* <= 2 L ||x_0 - x*||^2 / (k+1)^2, and the limit is a fixed point
    of the proximal-gradient map."""
    C, X, Y = small_problem(53, B=2, nx=6, ny=6)
    lam, tv, N = 0.05, "itv2d", 1500
    L = orc.lipschitz(C)
    xs, _ = orc.fista_tv(Y, C, lam, 400, N, tv=tv)
    Fs = objective(Y, C, xs, lam, tv)
    x0 = orc.adjoint(C, Y)
    R2 = ((x0 - xs) ** 2).sum()
    for k in (1, 2, 4, 8, 16, 32):
        xk, _ = orc.fista_tv(Y, C, lam, k, N, tv=tv)
        assert objective(Y, C, xk, lam, tv) - Fs <= 2 * L * R2 / (k + 1) ** 2 + 1e-9
    z = xs + orc.adjoint(C, (Y - orc.forward(C, xs)) / L)
    assert np.abs(orc.tv_denoise(z, lam / L, N, tv) - xs).max() < 1e-5


def test_twist_and_fista_reach_the_same_objective():
    """Two different iterations on the same convex objective: their limits
    have the same value (the minimiser need not be unique when Phi has a null
    space), and that value is below the starting point's."""
    C, X, Y = small_problem(54, B=2, nx=6, ny=7)
    lam, tv = 0.05, "atv"
    xf, _ = orc.fista_tv(Y, C, lam, 600, 800, tv=tv)
    xt, _ = orc.twist_tv(Y, C, lam, 600, 800, tv=tv)
    Ff, Ft = objective(Y, C, xf, lam, tv), objective(Y, C, xt, lam, tv)
    assert abs(Ff - Ft) <= 1e-6 * Ff
    assert Ff < objective(Y, C, orc.adjoint(C, Y), lam, tv)


def test_twist_default_parameters():
    a, b = orc.twist_default_ab(1e-4, 1.0)
    rho = (1 - 0.01) / (1 + 0.01)
    assert abs(a - (1 + rho ** 2)) < 1e-15 and abs(b - 2 * a / 1.0001) < 1e-15
    assert 0 < a < 2 and 0 < b < 2 * a  # the convergence range of TwIST for spectrum bound 1
    C = np.zeros((2, 3, 3))
    with pytest.raises(ValueError):
        orc.fista_tv(np.zeros((3, 3)), C, 0.1, 2, 2)


# ---------------------------------------------------------------------------
# ATV-Clip (Sec. 2.3, Algorithm 1): per-direction iterative clipping.
# ---------------------------------------------------------------------------

def tv1d_prox_rows(X, T):
    """prox of T ||D x||_1 along the last axis, row by row, through the box-
    constrained dual min 1/2 ||x - D^T w||^2, |w| <= T, solved by scipy's
    L-BFGS-B (an independent solver)."""
    n = X.shape[-1]
    D = diff_matrix(n)
    out = np.empty_like(X)
    for idx in np.ndindex(X.shape[:-1]):
        x = X[idx]
        if n == 1:
            out[idx] = x
            continue

        def f(w):
            r = x - D.T @ w
            return 0.5 * r @ r, -(D @ r)
        res = scipy.optimize.minimize(f, np.zeros(n - 1), jac=True, method="L-BFGS-B",
                                      bounds=[(-T, T)] * (n - 1), options={"ftol": 1e-15, "gtol": 1e-12,
                                                                           "maxiter": 10000})
        out[idx] = x - D.T @ res.x
    return out


def test_clip_first_step_closed_form():
    x = rng(60).uniform(size=(2, 5, 6))
    lam, alpha = 0.02, 4.0
    g = dense_grad(x)
    w1 = np.clip(g / alpha, -2 * lam, 2 * lam)
    th, w = orc.clip_denoise(x, lam, 1, alpha, return_dual=True)
    np.testing.assert_allclose(w, w1, rtol=0, atol=1e-15)
    np.testing.assert_allclose(th, x - dense_grad_adj(w1), rtol=0, atol=1e-15)


def test_clip_converges_to_sum_of_directional_1d_proxes():
    """The h and v duals never interact: the limit is
    prox_{2 lam TV_h}(x) + prox_{2 lam TV_v}(x) - x, each a family of 1-D TV
    proxes (rows, resp. columns) with weight 2 lam."""
    x = rng(61).uniform(size=(2, 7, 9))
    lam = 0.05
    th = orc.clip_denoise(x, lam, 20000, 4.0)
    h = tv1d_prox_rows(x, 2 * lam)
    v = np.swapaxes(tv1d_prox_rows(np.swapaxes(x, 1, 2), 2 * lam), 1, 2)
    np.testing.assert_allclose(th, h + v - x, rtol=0, atol=1e-6)


def test_clip_large_lambda_gives_row_plus_column_means():
    """A threshold larger than any dual the 1-D problems need: each 1-D prox
    is the mean of its row (column), so theta = row mean + column mean - x."""
    x = rng(62).uniform(size=(2, 5, 6))
    th = orc.clip_denoise(x, 50.0, 5000, 4.0)
    ref = x.mean(axis=2, keepdims=True) + x.mean(axis=1, keepdims=True) - x
    np.testing.assert_allclose(th, ref, rtol=0, atol=1e-9)


def test_clip_inside_gap():
    """GAP with the Clip denoiser: the outer loop passes the denoiser input and
    carries nothing else (written-out loop), and the measurement holds."""
    C, X, Y = small_problem(63, B=3, nx=8, ny=9)
    x, th = orc.gap_tv(Y, C, 0.05, 3, 6, tv="atv", clip=True, clip_alpha=5.0)
    S = orc.weights(C)
    t = orc.adjoint(C, Y)
    for _ in range(3):
        xe = t + orc.adjoint(C, (Y - orc.forward(C, t)) * S)
        t = orc.clip_denoise(xe, 0.05, 6, 5.0)
    np.testing.assert_allclose(x, xe, rtol=0, atol=1e-14)
    np.testing.assert_allclose(th, t, rtol=0, atol=1e-14)
    with pytest.raises(ValueError):
        orc.gap_tv(Y, C, 0.05, 1, 2, tv="itv2d", clip=True)


# ---------------------------------------------------------------------------
# Outer frameworks on hand-worked examples (ADMM Eq. (24)-(26), FISTA
# Eq. (14)-(17), TwIST Eq. (18)-(20)) and the ADMM fixed point.
# ---------------------------------------------------------------------------

FRAMEWORKS = os.path.join(os.path.dirname(__file__), "golden", "framework_worked_examples.json")


def framework_case(name):
    return next(c for c in json.load(open(FRAMEWORKS))["cases"] if c["name"] == name)


def exact(values):
    """Golden entries are exact rationals written as strings, or decimals."""
    from fractions import Fraction
    return np.array([float(Fraction(v)) if isinstance(v, str) else float(v) for v in values])


def test_golden_admm_three_iterations():
    """Pins the multiplier update u <- u + x - theta and the denoiser input
    u + x: u is nonzero from the first iteration on and changes x^(2), x^(3)."""
    g = framework_case("admm_atv_1x3_three_iterations")
    C, Y = np.array(g["C"]), np.array(g["Y"])
    for T, ref in g["by_T"].items():
        x, th = orc.admm_tv(Y, C, g["lam"], g["rho"], int(T), g["n_inner"], tv=g["tv"])
        np.testing.assert_allclose(x[0, 0], exact(ref["x"]), rtol=0, atol=1e-15)
        np.testing.assert_allclose(th[0, 0], exact(ref["theta"]), rtol=0, atol=1e-15)


def test_golden_fista_three_iterations():
    """Pins the tau sequence and the direction of the extrapolation (a pixel
    with c^2 = L/4 keeps moving, so the momentum shows in theta^(3))."""
    g = framework_case("fista_identity_denoiser_1x2")
    C, Y = np.array(g["C"]), np.array(g["Y"])
    for T, ref in g["by_T"].items():
        x, th = orc.fista_tv(Y, C, g["lam"], int(T), g["n_inner"], tv=g["tv"])
        np.testing.assert_allclose(x[0, 0], exact(ref["x"]), rtol=0, atol=2e-15)
        np.testing.assert_allclose(th[0, 0], exact(ref["theta_next"]), rtol=0, atol=2e-15)


def test_golden_twist_three_iterations():
    """Pins the two-step weights (1 - alpha) on x^(t-1), (alpha - beta) on
    x^(t) with alpha != 1, and the start x^(1) = theta^(0)."""
    g = framework_case("twist_identity_denoiser_1x2")
    C, Y = np.array(g["C"]), np.array(g["Y"])
    for T, ref in g["by_T"].items():
        x, th = orc.twist_tv(Y, C, g["lam"], int(T), g["n_inner"], tv=g["tv"], alpha=g["alpha"], beta=g["beta"])
        np.testing.assert_allclose(x[0, 0], exact(ref["x"]), rtol=0, atol=1e-15)
        np.testing.assert_allclose(th[0, 0], exact(ref["theta"]), rtol=0, atol=1e-15)


def dense_difference_rows(B, nx, ny):
    """Every difference of Eq. (7) as a row acting on vec_video (one +1, one -1)."""
    rows = []
    for k in range(B):
        for i in range(nx):
            for j in range(ny):
                for di, dj in ((0, 1), (1, 0)):
                    if i + di < nx and j + dj < ny:
                        e = np.zeros((B, nx, ny))
                        e[k, i + di, j + dj] = 1.0
                        e[k, i, j] = -1.0
                        rows.append(vec_video(e))
    return np.array(rows)


def test_admm_converges_to_penalised_least_squares_minimiser():
    """Scaled ADMM for min f(x) + g(theta), x = theta, alternates
    x = argmin f + rho/2 ||x - theta + u||^2, theta = prox_{g/rho}(x + u),
    u += x - theta. The denoiser solves prox_{lambda TV}, so g = rho lambda TV
    and the limit minimises 1/2 ||y - Phi x||^2 + rho lambda ATV(x). That
    minimum is computed independently by scipy's SLSQP on the epigraph form
    (variables x, t; -t <= D x <= t; objective 1/2 ||y - Phi x||^2 +
    rho lambda sum t) with dense Phi and D, and compared by value (Phi has a
    null space, so the minimiser itself need not be unique)."""
    r = rng(7)
    B, nx, ny = 2, 3, 3
    C = (r.random((B, nx, ny)) < 0.6).astype(float)
    Y = orc.forward(C, r.random((B, nx, ny))) + 0.05 * r.standard_normal((nx, ny))
    lam, rho = 0.05, 2.0
    mu = rho * lam
    x, th = orc.admm_tv(Y, C, lam, rho, 500, 300, tv="atv")
    assert np.abs(x - th).max() < 1e-10  # consensus x = theta at the limit

    V = B * nx * ny
    Phi, Dm, yv = dense_phi(C), dense_difference_rows(B, nx, ny), Y.ravel(order="F")
    m = Dm.shape[0]

    def f(zv):
        res = yv - Phi @ zv[:V]
        return 0.5 * res @ res + mu * zv[V:].sum()

    def fgrad(zv):
        return np.concatenate([-Phi.T @ (yv - Phi @ zv[:V]), mu * np.ones(m)])

    A = np.block([[Dm, np.eye(m)], [-Dm, np.eye(m)]])
    x0 = vec_video(orc.adjoint(C, Y))
    res = scipy.optimize.minimize(f, np.concatenate([x0, np.abs(Dm @ x0)]), jac=fgrad, method="SLSQP",
                                  constraints=[{"type": "ineq", "fun": lambda z: A @ z, "jac": lambda z: A}],
                                  options={"ftol": 1e-15, "maxiter": 2000})
    assert res.success

    def F(vol):
        xv = vec_video(vol)
        rr = yv - Phi @ xv
        return 0.5 * rr @ rr + mu * np.abs(Dm @ xv).sum()

    assert abs(F(x) - res.fun) <= 1e-9 * res.fun
