"""GPU parity: every entry point of the C ABI against the FP64 oracle.

Inputs come from the seeded generator (scene, masks, noise); the measurement
Y is formed by the oracle in FP64 and rounded once to float32, and both sides
consume exactly those float32 arrays. Floating-point results are compared by
relative L2 error (bar 1e-4) and PSNR difference (bar 0.01 dB); results that
the oracle cannot produce at full size are checked through properties that
hold at any size.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import oracle as orc  # noqa: E402
from paper_2005_08028_amd import synth  # noqa: E402

REL_TOL = 1e-4
PSNR_TOL = 0.01


def f32(v):
    """The C ABI takes lambda and rho as float32; the oracle gets the same values."""
    return float(np.float32(v))


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


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().float().cpu().numpy().astype(np.float64)


def rel_l2(a, ref):
    n = np.linalg.norm(ref)
    return np.linalg.norm(a - ref) / (n if n > 0 else 1.0)


def say(*a):
    print(*a, flush=True)


# ---------------------------------------------------------------------------
# Sensing operator.
# ---------------------------------------------------------------------------

SHAPES = [(1, 1, 1), (2, 3, 70), (8, 17, 255), (3, 130, 129), (8, 256, 256)]


@pytest.mark.parametrize("B,nx,ny", SHAPES)
def test_forward_adjoint(sc, ctx, B, nx, ny):
    r = np.random.default_rng(nx * 1000 + ny)
    C = synth.masks_bernoulli(r, nx, ny, B)
    X = r.uniform(size=(B, nx, ny)).astype(np.float32)
    Yv = r.uniform(size=(nx, ny)).astype(np.float32)
    Y = host(sc.sci_forward(ctx, dev(C), dev(X)))
    assert rel_l2(Y, orc.forward(C, X)) < 1e-6
    Xa = host(sc.sci_adjoint(ctx, dev(C), dev(Yv)))
    np.testing.assert_array_equal(Xa, orc.adjoint(C, Yv).astype(np.float32))
    lhs = (Y * Yv).sum()
    rhs = (X.astype(np.float64) * Xa).sum()
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs) + 1e-6


# ---------------------------------------------------------------------------
# TV denoiser.
# ---------------------------------------------------------------------------

DEN_SHAPES = [(1, 1, 1), (1, 2, 2), (2, 5, 3), (3, 17, 63), (2, 33, 125), (4, 130, 64), (9, 20, 70), (24, 16, 64)]


@pytest.mark.parametrize("tv,schedule", [("atv", "stream"), ("itv2d", "stream"), ("vtv", "stream"),
                                         ("atv", "fused"), ("itv2d", "fused")])
@pytest.mark.parametrize("B,nx,ny", DEN_SHAPES)
def test_denoise_matches_oracle(sc, ctx, tv, schedule, B, nx, ny):
    r = np.random.default_rng(B * 7 + nx * 13 + ny)
    x = r.uniform(size=(B, nx, ny)).astype(np.float32)
    for n, accel in ((1, True), (2, True), (7, True), (5, False)):
        prm = sc.tv_params(tv=tv, lam=0.1, n_inner=n, accel=accel, schedule=schedule)
        dual = torch.empty((2, B, nx, ny), device="cuda")
        th, _, its, st = sc.sci_tv_denoise(ctx, dev(x), prm, dual_out=dual)
        ref, pref = orc.tv_denoise(x, f32(0.1), n, tv, accel=accel, return_dual=True)
        e = rel_l2(host(th), ref)
        ep = np.abs(host(dual) - pref).max()
        say(f"denoise {tv}/{schedule} B={B} {nx}x{ny} N={n} accel={accel}: rel-L2 {e:.2e}, dual max-abs {ep:.2e}")
        assert its == n
        assert e <= REL_TOL
        assert ep <= 1e-4


# VTV splits a pixel's frames over up to 8 wavefronts: 3 and 4 frames per
# wavefront, and splits whose last wavefront holds spare slots (17 = 6 x 3 - 1,
# 29 = 8 x 4 - 3); several strips and row segments
@pytest.mark.parametrize("dt", ["f32", "bf16"])
@pytest.mark.parametrize("B,nx,ny", [(17, 70, 33), (29, 9, 130), (32, 40, 70), (10, 100, 125)])
def test_vtv_frame_groups(sc, ctx, B, nx, ny, dt):
    r = np.random.default_rng(B * 11 + nx + ny)
    x = r.uniform(size=(B, nx, ny)).astype(np.float32)
    for n in (3, 6):
        prm = sc.tv_params(tv="vtv", lam=0.1, n_inner=n, schedule="stream", dual_dtype=dt)
        th, _, its, _ = sc.sci_tv_denoise(ctx, dev(x), prm)
        ref = orc.tv_denoise(x, f32(0.1), n, "vtv")
        e = rel_l2(host(th), ref)
        say(f"vtv frame groups B={B} {nx}x{ny} {dt} N={n}: rel-L2 {e:.2e}")
        assert its == n
        # 16-bit storage: the per-store rounding bound 4 lambda u per iteration
        assert e <= (REL_TOL if dt == "f32" else 2e-2)


FUSED_SHAPES = [(1, 1, 1), (2, 3, 2), (1, 5, 300), (3, 250, 130), (2, 118, 54), (2, 117, 53), (1, 240, 107)]


@pytest.mark.parametrize("tv", ["atv", "itv2d"])
@pytest.mark.parametrize("B,nx,ny", FUSED_SHAPES)
def test_fused_schedule_bitwise_equals_streaming(sc, ctx, tv, B, nx, ny):
    """The tiled multi-iteration passes evaluate the same per-voxel
    expressions as one-pass-per-iteration streaming: identical bits with
    float32 dual storage, for every pass split (N = 1..13), with and without
    momentum, cold and warm starts. With 16-bit storage the fused schedule
    rounds the dual only between passes (float32 registers inside a pass), so
    both schedules are held to the mixed-precision bound against the oracle
    instead, the fused one being no less accurate."""
    r = np.random.default_rng(nx * 31 + ny + B)
    x = dev(r.uniform(size=(B, nx, ny)).astype(np.float32))
    p0 = orc.project_dual(r.normal(size=(2, B, nx, ny)), tv).astype(np.float32)
    cases = [(n, True, False, "f32") for n in (1, 2, 3, 4, 5, 6, 7, 10, 13)]
    cases += [(5, False, False, "f32"), (7, True, True, "f32"), (9, True, False, "bf16"), (8, True, True, "f16")]
    for n, accel, warm, dt in cases:
        outs = []
        for schedule in ("stream", "fused"):
            prm = sc.tv_params(tv=tv, lam=0.1, n_inner=n, accel=accel, schedule=schedule, dual_dtype=dt)
            ddt = sc.DUAL_TORCH[prm.dual_dtype]
            dual = torch.empty((2, B, nx, ny), device="cuda", dtype=ddt)
            init = dev(p0, ddt) if warm else None
            th, _, _, _ = sc.sci_tv_denoise(ctx, x, prm, dual_init=init, dual_out=dual)
            outs.append((host(th), host(dual)))
        if dt == "f32":
            np.testing.assert_array_equal(outs[0][0], outs[1][0], err_msg=f"theta N={n} accel={accel} warm={warm}")
            np.testing.assert_array_equal(outs[0][1], outs[1][1], err_msg=f"dual N={n} accel={accel} warm={warm}")
        else:
            ref = orc.tv_denoise(x.cpu().numpy(), f32(0.1), n, tv, accel=accel, p_init=p0 if warm else None)
            u = 2.0 ** -8 if dt == "bf16" else 2.0 ** -11
            e_s, e_f = np.abs(outs[0][0] - ref).max(), np.abs(outs[1][0] - ref).max()
            assert e_s <= 10 * 4 * 0.1 * u and e_f <= 10 * 4 * 0.1 * u, (e_s, e_f)
            assert e_f <= 1.5 * e_s + 1e-6, (e_s, e_f)


@pytest.mark.parametrize("tv", ["atv", "itv2d"])
def test_every_tile_shape_gives_identical_bits(sc, ctx, tv):
    r = np.random.default_rng(17)
    for B, nx, ny in ((2, 200, 150), (1, 33, 70)):
        x = dev(r.uniform(size=(B, nx, ny)).astype(np.float32))
        ref = None
        for shape in range(1, sc.sci_tile_shape_count() + 1):
            prm = sc.tv_params(tv=tv, lam=0.1, n_inner=10, schedule="fused", tile_shape=shape)
            th, _, _, _ = sc.sci_tv_denoise(ctx, x, prm)
            th = host(th)
            if ref is None:
                ref = th
            np.testing.assert_array_equal(th, ref, err_msg=f"shape {shape} {sc.sci_tile_shape_info(shape)}")
        best, passes, times = sc.sci_autotune(ctx, x, sc.tv_params(tv=tv, lam=0.1, n_inner=10))
        assert 1 <= best <= sc.sci_tile_shape_count() and 1 <= passes <= 3
        assert all(t > 0 for row in times for t in row)
        for np_ in (1, 2, 3, 10):
            prm = sc.tv_params(tv=tv, lam=0.1, n_inner=10, schedule="fused", tile_passes=np_)
            th, _, _, _ = sc.sci_tv_denoise(ctx, x, prm)
            np.testing.assert_array_equal(host(th), ref, err_msg=f"{np_} passes")
        th, _, _, _ = sc.sci_tv_denoise(ctx, x, sc.tv_params(tv=tv, lam=0.1, n_inner=10))
        np.testing.assert_array_equal(host(th), ref)


def row_shapes(sc):
    return [k for k in range(1, sc.sci_tile_shape_count() + 1) if sc.sci_tile_shape_pipelined(k)]


# several row segments per frame (segment heights 32 .. 256), ragged strips,
# images narrower than one strip and shorter than the pipeline fill
ROW_CASES = [(1, 1, 1), (2, 3, 2), (1, 5, 300), (2, 300, 130), (1, 97, 214), (3, 70, 107)]


@pytest.mark.parametrize("tv", ["atv", "itv2d"])
@pytest.mark.parametrize("B,nx,ny", ROW_CASES)
def test_row_pipelined_bitwise_equals_streaming(sc, ctx, tv, B, nx, ny):
    """Row-pipelined shapes against one-pass-per-iteration streaming, float32
    duals: pass lengths 1..10, one pass and several (the later passes start
    from the previous pass's p and p_prev), cold and warm starts, momentum on
    and off, final dual returned: identical bits for theta and the dual."""
    shapes = row_shapes(sc)
    assert shapes
    r = np.random.default_rng(nx * 7 + ny * 3 + B)
    x = dev(r.uniform(size=(B, nx, ny)).astype(np.float32))
    p0 = dev(orc.project_dual(r.normal(size=(2, B, nx, ny)), tv).astype(np.float32))
    cases = [(1, 1, True, False), (2, 1, True, True), (3, 1, False, False), (6, 1, True, False),
             (9, 1, True, True), (10, 1, True, False), (10, 2, True, True), (13, 2, True, False),
             (20, 3, False, True), (5, 5, True, False)]
    for n, passes, accel, warm in cases:
        init = p0 if warm else None
        prm = sc.tv_params(tv=tv, lam=0.1, n_inner=n, accel=accel, schedule="stream")
        dref = torch.empty((2, B, nx, ny), device="cuda")
        tref, _, _, _ = sc.sci_tv_denoise(ctx, x, prm, dual_init=init, dual_out=dref)
        tref, dref = host(tref), host(dref)
        for k in shapes:
            prm = sc.tv_params(tv=tv, lam=0.1, n_inner=n, accel=accel, schedule="fused", tile_shape=k,
                               tile_passes=passes)
            d = torch.empty((2, B, nx, ny), device="cuda")
            th, _, its, _ = sc.sci_tv_denoise(ctx, x, prm, dual_init=init, dual_out=d)
            msg = f"shape {k} {sc.sci_tile_shape_info(k)} N={n} passes={passes} accel={accel} warm={warm}"
            assert its == n, msg
            np.testing.assert_array_equal(host(th), tref, err_msg="theta " + msg)
            np.testing.assert_array_equal(host(d), dref, err_msg="dual " + msg)
    say(f"row-pipelined {tv} B={B} {nx}x{ny}: {len(cases)} cases x {len(shapes)} shapes bit-identical")


# 1..4 frames per wavefront (B = 8, 10, 24, 32 and splits with spare slots:
# 3, 17, 29; B = 16 takes 10-level passes at 2 frames per wavefront), several
# row segments, ragged strips, tiny images
VTV_FUSED_CASES = [(1, 1, 1), (3, 2, 5), (8, 70, 33), (10, 130, 150), (16, 40, 70), (17, 45, 100), (24, 64, 64),
                   (29, 9, 130), (32, 40, 70)]


@pytest.mark.parametrize("B,nx,ny", VTV_FUSED_CASES)
def test_vtv_fused_bitwise_equals_streaming(sc, ctx, B, nx, ny):
    """Row-pipelined VTV against one-pass-per-iteration streaming VTV, float32
    duals: one pass and several (pass lengths up to the kernel's limit for the
    frames per wavefront), cold and warm starts, momentum on and off, final
    dual returned: identical bits for theta and the dual."""
    r = np.random.default_rng(B * 13 + nx + ny)
    x = dev(r.uniform(size=(B, nx, ny)).astype(np.float32))
    p0 = dev(orc.project_dual(r.normal(size=(2, B, nx, ny)), "vtv").astype(np.float32))
    cases = [(1, 0, True, False), (2, 0, True, True), (4, 0, False, False), (5, 0, True, False),
             (7, 0, True, True), (10, 0, True, False), (10, 5, True, True), (13, 0, False, True)]
    for n, passes, accel, warm in cases:
        init = p0 if warm else None
        outs = []
        for schedule in ("stream", "fused"):
            prm = sc.tv_params(tv="vtv", lam=0.1, n_inner=n, accel=accel, schedule=schedule, tile_passes=passes)
            d = torch.empty((2, B, nx, ny), device="cuda")
            th, _, its, _ = sc.sci_tv_denoise(ctx, x, prm, dual_init=init, dual_out=d)
            assert its == n
            outs.append((host(th), host(d)))
        msg = f"VTV B={B} {nx}x{ny} N={n} passes={passes} accel={accel} warm={warm}"
        np.testing.assert_array_equal(outs[1][0], outs[0][0], err_msg="theta " + msg)
        np.testing.assert_array_equal(outs[1][1], outs[0][1], err_msg="dual " + msg)
    ref = orc.tv_denoise(x.cpu().numpy(), f32(0.1), 10, "vtv")
    th, _, _, _ = sc.sci_tv_denoise(ctx, x, sc.tv_params(tv="vtv", lam=0.1, n_inner=10))
    assert rel_l2(host(th), ref) <= REL_TOL
    say(f"VTV fused B={B} {nx}x{ny}: {len(cases)} cases bit-identical to streaming")


def test_vtv_fused_every_frame_split(sc, ctx):
    """Frame counts across every split of the fused VTV kernel (1..4 frames
    per wavefront, last wavefront full or with spare slots): the fused bits
    equal the streaming ones for a single pass and for a warm two-pass call."""
    r = np.random.default_rng(81)
    for B in (1, 2, 5, 7, 8, 9, 11, 15, 16, 17, 20, 23, 24, 25, 28, 31, 32):
        x = dev(r.uniform(size=(B, 21, 70)).astype(np.float32))
        p0 = dev(orc.project_dual(r.normal(size=(2, B, 21, 70)), "vtv").astype(np.float32))
        for n, warm in ((3, False), (7, True)):
            init = p0 if warm else None
            outs = []
            for schedule in ("stream", "fused"):
                prm = sc.tv_params(tv="vtv", lam=0.1, n_inner=n, schedule=schedule)
                d = torch.empty((2, B, 21, 70), device="cuda")
                th, _, _, _ = sc.sci_tv_denoise(ctx, x, prm, dual_init=init, dual_out=d)
                outs.append((host(th), host(d)))
            np.testing.assert_array_equal(outs[1][0], outs[0][0], err_msg=f"theta B={B} N={n} warm={warm}")
            np.testing.assert_array_equal(outs[1][1], outs[0][1], err_msg=f"dual B={B} N={n} warm={warm}")


@pytest.mark.parametrize("B", [3, 10, 24])
def test_vtv_16bit_cold_single_pass(sc, ctx, B):
    """16-bit VTV storage in one cold pass: the dual is held in float32
    registers for the whole pass, so theta is the float32 fused result bit
    for bit, and the dual returned in 16 bits is the float32 dual rounded to
    nearest even (torch's conversion), also bit for bit."""
    r = np.random.default_rng(B * 23)
    x = dev(r.uniform(size=(B, 90, 140)).astype(np.float32))
    n = 4
    d32 = torch.empty((2, B, 90, 140), device="cuda")
    ref = host(sc.sci_tv_denoise(ctx, x, sc.tv_params(tv="vtv", lam=0.1, n_inner=n, schedule="fused"),
                                 dual_out=d32)[0])
    for dt in ("bf16", "f16"):
        th = host(sc.sci_tv_denoise(ctx, x, sc.tv_params(tv="vtv", lam=0.1, n_inner=n, dual_dtype=dt))[0])
        np.testing.assert_array_equal(th, ref, err_msg=dt)
        ddt = sc.DUAL_TORCH[sc.DUAL[dt]]
        d = torch.empty((2, B, 90, 140), device="cuda", dtype=ddt)
        th_d = host(sc.sci_tv_denoise(ctx, x, sc.tv_params(tv="vtv", lam=0.1, n_inner=n, dual_dtype=dt), dual_out=d)[0])
        np.testing.assert_array_equal(th_d, ref, err_msg=dt + " with the dual returned")
        assert torch.equal(d.view(torch.int16), d32.to(ddt).view(torch.int16)), dt + " dual rounding"


@pytest.mark.parametrize("solver", ["gap", "admm"])
def test_vtv_fused_solvers_bitwise(sc, ctx, solver):
    """Whole GAP / ADMM VTV solves, with and without the warm dual, eager and
    graph-launched: the fused schedule gives the bits of the streaming one."""
    pr = synth.make_problem(120, 100, 10, seed=31, sigma=0.01)
    Y = orc.measurement(pr.masks, pr.truth, pr.noise)
    for warm in (False, True):
        kw = dict(outer_iters=4, rho=0.01, tv="vtv", lam=0.1, n_inner=6, warm_dual=warm)
        xs, ts = run_solver(sc, ctx, solver, Y, pr.masks, schedule="stream", **kw)
        xf, tf = run_solver(sc, ctx, solver, Y, pr.masks, schedule="fused", **kw)
        np.testing.assert_array_equal(xf, xs, err_msg=f"{solver} warm={warm}")
        np.testing.assert_array_equal(tf, ts, err_msg=f"{solver} warm={warm}")
        for rep in range(2):
            xg, tg = run_solver(sc, ctx, solver, Y, pr.masks, schedule="fused", use_graph=True, **kw)
            _ = torch.ones(1000, device="cuda").sum().item()  # unrelated eager work between replays
            np.testing.assert_array_equal(xg, xs, err_msg=f"{solver} warm={warm} graph replay {rep}")


@pytest.mark.parametrize("tv", ["atv", "itv2d"])
def test_row_pipelined_matches_oracle(sc, ctx, tv):
    """Every row-pipelined shape against the FP64 oracle directly (several
    segments and strips, a ragged last strip), theta and the final dual."""
    B, nx, ny = 2, 300, 230
    r = np.random.default_rng(61)
    x = r.uniform(size=(B, nx, ny)).astype(np.float32)
    ref, pref = orc.tv_denoise(x, f32(0.1), 10, tv, return_dual=True)
    for k in row_shapes(sc):
        prm = sc.tv_params(tv=tv, lam=0.1, n_inner=10, schedule="fused", tile_shape=k, tile_passes=1)
        dual = torch.empty((2, B, nx, ny), device="cuda")
        th, _, _, _ = sc.sci_tv_denoise(ctx, dev(x), prm, dual_out=dual)
        e = rel_l2(host(th), ref)
        ep = np.abs(host(dual) - pref).max()
        say(f"row shape {k} {sc.sci_tile_shape_info(k)} {tv}: rel-L2 {e:.2e}, dual max-abs {ep:.2e}")
        assert e <= REL_TOL and ep <= 1e-4


@pytest.mark.parametrize("tv", ["atv", "itv2d"])
def test_row_pipelined_16bit_cold_pass(sc, ctx, tv):
    """A cold single pass that does not return the dual never stores it, so
    with 16-bit storage the row-pipelined shapes give the float32 bits, which
    are also those of the 16-bit default tile (float32 registers)."""
    r = np.random.default_rng(71)
    x = dev(r.uniform(size=(3, 150, 140)).astype(np.float32))
    ref = host(sc.sci_tv_denoise(ctx, x, sc.tv_params(tv=tv, lam=0.1, n_inner=10, schedule="fused",
                                                      tile_shape=1, tile_passes=1, dual_dtype="bf16"))[0])
    for dt in ("f32", "bf16", "f16"):
        for k in row_shapes(sc):
            prm = sc.tv_params(tv=tv, lam=0.1, n_inner=10, schedule="fused", tile_shape=k, tile_passes=1,
                               dual_dtype=dt)
            np.testing.assert_array_equal(host(sc.sci_tv_denoise(ctx, x, prm)[0]), ref, err_msg=f"{dt} shape {k}")


@pytest.mark.parametrize("solver", ["gap", "admm"])
def test_row_pipelined_solvers_bitwise(sc, ctx, solver):
    """Whole GAP / ADMM solves (ADMM takes u = s - theta from the kernel),
    with and without the warm dual across outer iterations: a row-pipelined
    shape gives the bits of the streaming schedule."""
    pr = synth.make_problem(150, 90, 6, seed=21, sigma=0.01)
    Y = orc.measurement(pr.masks, pr.truth, pr.noise)
    for warm in (False, True):
        kw = dict(outer_iters=4, rho=0.01, tv="itv2d", lam=0.1, n_inner=7, warm_dual=warm)
        xs, ts = run_solver(sc, ctx, solver, Y, pr.masks, schedule="stream", **kw)
        for k in row_shapes(sc):
            x, t = run_solver(sc, ctx, solver, Y, pr.masks, schedule="fused", tile_shape=k, **kw)
            np.testing.assert_array_equal(x, xs, err_msg=f"{solver} warm={warm} shape {k}")
            np.testing.assert_array_equal(t, ts, err_msg=f"{solver} warm={warm} shape {k}")


@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_denoise_default_schedule_matches_oracle(sc, ctx, tv):
    x = np.random.default_rng(3).uniform(size=(6, 70, 150)).astype(np.float32)
    prm = sc.tv_params(tv=tv, lam=0.07, n_inner=10)
    th, _, _, _ = sc.sci_tv_denoise(ctx, dev(x), prm)
    ref = orc.tv_denoise(x, f32(0.07), 10, tv)
    assert rel_l2(host(th), ref) <= REL_TOL


@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_denoise_warm_start(sc, ctx, tv):
    r = np.random.default_rng(4)
    x = r.uniform(size=(3, 40, 90)).astype(np.float32)
    p0 = orc.project_dual(r.normal(size=(2, 3, 40, 90)), tv)
    p0[0, :, :, -1] = 0.0
    p0[1, :, -1, :] = 0.0
    p0 = p0.astype(np.float32)
    prm = sc.tv_params(tv=tv, lam=0.1, n_inner=6)
    th, _, _, _ = sc.sci_tv_denoise(ctx, dev(x), prm, dual_init=dev(p0))
    ref = orc.tv_denoise(x, f32(0.1), 6, tv, p_init=p0)
    assert rel_l2(host(th), ref) <= REL_TOL


@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_denoise_special_cases(sc, ctx, tv):
    x = np.random.default_rng(5).uniform(size=(4, 31, 77)).astype(np.float32)
    for prm in (sc.tv_params(tv=tv, lam=0.0, n_inner=5), sc.tv_params(tv=tv, lam=0.1, n_inner=0)):
        th, _, _, _ = sc.sci_tv_denoise(ctx, dev(x), prm)
        np.testing.assert_array_equal(host(th), x)
    c = np.full((4, 31, 77), 0.37, np.float32)
    th, _, _, _ = sc.sci_tv_denoise(ctx, dev(c), sc.tv_params(tv=tv, lam=0.1, n_inner=8))
    np.testing.assert_array_equal(host(th), c)
    # lambda -> infinity: per-frame means
    xs = np.random.default_rng(6).uniform(size=(3, 8, 8)).astype(np.float32)
    th, _, _, _ = sc.sci_tv_denoise(ctx, dev(xs), sc.tv_params(tv=tv, lam=50.0, n_inner=3000))
    means = xs.astype(np.float64).mean(axis=(1, 2), keepdims=True)
    assert np.abs(host(th) - means).max() < 1e-4


@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_dual_gap_matches_oracle(sc, ctx, tv):
    x = np.random.default_rng(7).uniform(size=(5, 45, 66)).astype(np.float32)
    dual = torch.empty((2, 5, 45, 66), device="cuda")
    _, g_rel, _, _ = sc.sci_tv_denoise(ctx, dev(x), sc.tv_params(tv=tv, lam=0.1, n_inner=12), dual_out=dual,
                                       want_gap=True)
    p = host(dual)
    g_or, prim_or = orc.dual_gap(x, p, f32(0.1), tv)
    g_gpu, prim_gpu = sc.sci_dual_gap(ctx, dev(x), dual, tv, 0.1)
    assert abs(g_gpu - g_or) <= 1e-9 * prim_or
    assert abs(prim_gpu - prim_or) <= 1e-10 * prim_or
    assert abs(g_rel - g_or / prim_or) <= 1e-9
    # constant input: TV = 0, gap = 0
    c = np.full((2, 9, 9), 0.5, np.float32)
    g0, p0 = sc.sci_dual_gap(ctx, dev(c), torch.zeros((2, 2, 9, 9), device="cuda"), tv, 0.1)
    assert g0 == 0.0 and p0 == 0.0


# frames split over wavefronts (1..4 per wavefront for VTV, frame groups
# along the grid for the per-voxel TVs), several strips and row segments,
# ragged edges, single-row and single-column images
GAP_SHAPES = [(1, 9, 9), (8, 70, 130), (24, 33, 200), (10, 130, 64), (32, 20, 63), (3, 300, 17), (12, 17, 1),
              (5, 1, 40)]


@pytest.mark.parametrize("shape", GAP_SHAPES)
@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_dual_gap_shapes(sc, ctx, tv, shape):
    rng = np.random.default_rng(sum(shape))
    x = rng.uniform(size=shape).astype(np.float32)
    p = rng.uniform(-1.0, 1.0, size=(2,) + shape).astype(np.float32)
    g_or, prim_or = orc.dual_gap(x, p, f32(0.1), tv)
    g1 = sc.sci_dual_gap(ctx, dev(x), dev(p), tv, 0.1)
    g2 = sc.sci_dual_gap(ctx, dev(x), dev(p), tv, 0.1)
    assert g1 == g2  # fixed summation order
    assert abs(g1[0] - g_or) <= 1e-9 * prim_or
    assert abs(g1[1] - prim_or) <= 1e-10 * prim_or
    # 16-bit storage: the oracle sees the stored (rounded) values
    for dt in (torch.bfloat16, torch.float16):
        pd = dev(p).to(dt)
        g_or16, prim_or16 = orc.dual_gap(x, host(pd.float()), f32(0.1), tv)
        g16, prim16 = sc.sci_dual_gap(ctx, dev(x), pd, tv, 0.1)
        assert abs(g16 - g_or16) <= 1e-9 * prim_or16
        assert abs(prim16 - prim_or16) <= 1e-10 * prim_or16


def test_dual_gap_vtv_frame_limit(sc, ctx):
    x = torch.zeros((49, 8, 8), device="cuda")
    with pytest.raises(sc.SciError):
        sc.sci_dual_gap(ctx, x, torch.zeros((2, 49, 8, 8), device="cuda"), "vtv", 0.1)


@pytest.mark.parametrize("B,nx,ny", [(33, 17, 70), (40, 30, 66), (48, 9, 130)])
def test_vtv_many_frames_streaming(sc, ctx, B, nx, ny):
    """VTV at 33 to 48 frames (5 or 6 frames in each of 8 wavefronts, the
    streaming schedule, which the automatic schedule picks beyond 32 frames):
    the denoiser (cold, warm, with and without momentum; theta and dual), its
    16-bit storage, the FP64 duality gap and a GAP solve, each against the
    oracle; the automatic and streaming schedules agree bit for bit."""
    r = np.random.default_rng(B + nx)
    x = r.uniform(size=(B, nx, ny)).astype(np.float32)
    p0 = orc.project_dual(0.3 * r.normal(size=(2, B, nx, ny)), "vtv").astype(np.float32)
    for n, accel, warm in ((1, True, False), (7, True, False), (6, False, True), (5, True, True)):
        outs = []
        for schedule in ("auto", "stream"):
            prm = sc.tv_params(tv="vtv", lam=0.1, n_inner=n, accel=accel, schedule=schedule)
            dual = torch.empty((2, B, nx, ny), device="cuda")
            th, _, its, _ = sc.sci_tv_denoise(ctx, dev(x), prm, dual_init=dev(p0) if warm else None, dual_out=dual)
            assert its == n
            outs.append((host(th), host(dual)))
        np.testing.assert_array_equal(outs[0][0], outs[1][0])
        np.testing.assert_array_equal(outs[0][1], outs[1][1])
        ref, pref = orc.tv_denoise(x, f32(0.1), n, "vtv", accel=accel, p_init=p0 if warm else None,
                                   return_dual=True)
        e, ep = rel_l2(outs[0][0], ref), np.abs(outs[0][1] - pref).max()
        say(f"vtv B={B} {nx}x{ny} N={n} accel={accel} warm={warm}: rel-L2 {e:.2e}, dual {ep:.2e}")
        assert e <= REL_TOL and ep <= 1e-4
        g, prim = sc.sci_dual_gap(ctx, dev(x), dev(outs[0][1]), "vtv", 0.1)
        g_or, prim_or = orc.dual_gap(x, outs[0][1], f32(0.1), "vtv")
        assert abs(g - g_or) <= 1e-9 * prim_or and abs(prim - prim_or) <= 1e-10 * prim_or
    th16, _, _, _ = sc.sci_tv_denoise(ctx, dev(x), sc.tv_params(tv="vtv", lam=0.1, n_inner=10, dual_dtype="bf16"))
    e16 = rel_l2(host(th16), orc.tv_denoise(x, f32(0.1), 10, "vtv"))
    say(f"vtv B={B} bf16 duals, 10 iterations: rel-L2 {e16:.2e}")
    assert e16 <= 2e-2
    pr = synth.make_problem(nx, ny, B, seed=B, sigma=0.01)
    Y = orc.measurement(pr.masks, pr.truth, pr.noise)
    xg, _ = run_solver(sc, ctx, "gap", Y, pr.masks, outer_iters=3, tv="vtv", lam=0.1, n_inner=5, warm_dual=True)
    xr, _ = orc.gap_tv(Y, pr.masks, f32(0.1), 3, 5, tv="vtv", warm_dual=True)
    eg = rel_l2(xg, xr)
    say(f"GAP-VTV B={B} 3 x 5 warm: rel-L2 {eg:.2e}")
    assert eg <= REL_TOL


@pytest.mark.parametrize("tv", ["itv2d", "vtv"])
def test_dual_gap_full_size(sc, ctx, tv):
    """The 1024x1024x24 measurement's back-projection and a dual after a few
    FGP iterations, against the oracle's FP64 gap."""
    pr = synth.problem_from_config("cacti_1024x24")
    C = dev(pr.masks)
    Y = sc.sci_forward(ctx, C, dev(pr.truth))
    x = sc.sci_adjoint(ctx, C, Y)
    dual = torch.empty((2,) + tuple(x.shape), device="cuda")
    sc.sci_tv_denoise(ctx, x, sc.tv_params(tv=tv, lam=0.1, n_inner=5), dual_out=dual)
    g_or, prim_or = orc.dual_gap(host(x), host(dual), f32(0.1), tv)
    g, prim = sc.sci_dual_gap(ctx, x, dual, tv, 0.1)
    say(f"{tv} 1024x1024x24: gap {g:.6e} (oracle {g_or:.6e}), primal {prim:.6e}")
    assert abs(g - g_or) <= 1e-9 * prim_or
    assert abs(prim - prim_or) <= 1e-10 * prim_or


@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_gap_controlled_denoise(sc, ctx, tv):
    x = np.random.default_rng(8).uniform(size=(4, 64, 64)).astype(np.float32)
    prm = sc.tv_params(tv=tv, lam=0.1, gap_tol=1e-4, n_inner_max=2000, gap_check_every=5)
    th, g, its, st = sc.sci_tv_denoise(ctx, dev(x), prm, want_gap=True)
    say(f"{tv}: gap<=1e-4 after {its} iterations (rel gap {g:.2e})")
    assert st == sc.SCI_OK and g <= 1e-4 and its % 5 == 0
    ref = orc.tv_denoise(x, f32(0.1), its, tv)
    assert rel_l2(host(th), ref) <= REL_TOL
    prm = sc.tv_params(tv=tv, lam=0.1, gap_tol=1e-12, n_inner_max=6, gap_check_every=4)
    _, _, its, st = sc.sci_tv_denoise(ctx, dev(x), prm, want_gap=True)
    assert st == sc.SCI_NOT_CONVERGED and its == 6


@pytest.mark.parametrize("dt,bound", [("f32", REL_TOL), ("bf16", 2e-2), ("f16", 3e-3)])
def test_gap_controlled_vtv_records(sc, ctx, dt, bound):
    """Gap-controlled VTV at B = 24: every 10 iterations between two gap
    checks run as two on-chip passes that hand the dual over as one record
    per voxel. float32: the streaming schedule's iterates bit for bit, to
    convergence. 16-bit: at most 30 iterations towards a tolerance of 1e-12
    (below what a 16-bit dual can certify: rounded to 16 bits it may leave the
    unit ball by half an ulp, and its gap can then come out at or below zero,
    which meets any tolerance), against the oracle within the storage type's
    bound, and the reported gap is the FP64 gap of the returned dual."""
    r = np.random.default_rng(24)
    B, nx, ny = 24, 40, 70
    x = r.uniform(size=(B, nx, ny)).astype(np.float32)
    ddt = sc.DUAL_TORCH[sc.DUAL[dt]]
    p0 = dev(orc.project_dual(0.3 * r.normal(size=(2, B, nx, ny)), "vtv").astype(np.float32), ddt)
    if dt == "f32":
        out = {}
        for schedule in ("stream", "auto"):
            prm = sc.tv_params(tv="vtv", lam=0.1, gap_tol=1e-4, n_inner_max=3000, gap_check_every=10,
                               schedule=schedule)
            dual = torch.empty((2, B, nx, ny), device="cuda")
            th, g, its, st = sc.sci_tv_denoise(ctx, dev(x), prm, dual_init=p0, dual_out=dual, want_gap=True)
            assert st == sc.SCI_OK and g <= 1e-4
            out[schedule] = (host(th), host(dual), its)
        say(f"vtv B=24 gap-controlled: {out['auto'][2]} iterations on both schedules")
        assert out["stream"][2] == out["auto"][2]
        np.testing.assert_array_equal(out["stream"][0], out["auto"][0])
        np.testing.assert_array_equal(out["stream"][1], out["auto"][1])
        its, th = out["auto"][2], out["auto"][0]
    else:
        prm = sc.tv_params(tv="vtv", lam=0.1, gap_tol=1e-12, n_inner_max=30, gap_check_every=10, dual_dtype=dt)
        dual = torch.empty((2, B, nx, ny), device="cuda", dtype=ddt)
        tht, g, its, st = sc.sci_tv_denoise(ctx, dev(x), prm, dual_init=p0, dual_out=dual, want_gap=True)
        say(f"vtv B=24 {dt} gap-controlled: status {st}, {its} iterations, rel gap {g:.3e}")
        assert its % 10 == 0 and 10 <= its <= 30
        assert (st == sc.SCI_NOT_CONVERGED and its == 30 and g > 1e-12) or (st == sc.SCI_OK and g <= 1e-12)
        th = host(tht)
        g64, prim = orc.dual_gap(x, host(dual), f32(0.1), "vtv")
        assert abs(g - g64 / prim) <= 1e-3 * abs(g64 / prim) + 1e-9
    ref = orc.tv_denoise(x, f32(0.1), its, "vtv", p_init=host(p0))
    e = rel_l2(th, ref)
    say(f"vtv B=24 {dt} gap-controlled, {its} iterations: rel-L2 {e:.2e}")
    assert e <= bound


@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_gap_controlled_schedules_agree(sc, ctx, tv):
    """Gap-controlled denoising: iterations between gap checks run as on-chip
    passes (auto) or one pass each (stream); same iterates bit for bit."""
    x = np.random.default_rng(10).uniform(size=(3, 70, 90)).astype(np.float32)
    p0 = np.random.default_rng(11).uniform(-0.5, 0.5, size=(2, 3, 70, 90)).astype(np.float32)
    out = {}
    for schedule in ("stream", "auto"):
        prm = sc.tv_params(tv=tv, lam=0.1, gap_tol=1e-4, n_inner_max=3000, gap_check_every=7, schedule=schedule)
        dual = torch.empty((2, 3, 70, 90), device="cuda")
        th, g, its, st = sc.sci_tv_denoise(ctx, dev(x), prm, dual_init=dev(p0), dual_out=dual, want_gap=True)
        out[schedule] = (host(th), host(dual), its, g)
    say(f"{tv}: gap-controlled {out['auto'][2]} iterations on both schedules")
    assert out["stream"][2] == out["auto"][2]
    np.testing.assert_array_equal(out["stream"][0], out["auto"][0])
    np.testing.assert_array_equal(out["stream"][1], out["auto"][1])
    ref = orc.tv_denoise(x, f32(0.1), out["auto"][2], tv, p_init=p0)
    assert rel_l2(out["auto"][0], ref) <= REL_TOL


@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
@pytest.mark.parametrize("B,nx,ny", [(1, 1, 1), (2, 5, 3), (3, 17, 63), (4, 130, 64), (9, 20, 70), (24, 16, 64)])
def test_chambolle04_matches_oracle(sc, ctx, tv, B, nx, ny):
    """Chambolle's (2004) semi-implicit step in place of the projection."""
    r = np.random.default_rng(B * 5 + nx * 3 + ny)
    x = r.uniform(size=(B, nx, ny)).astype(np.float32)
    p0 = r.uniform(-0.5, 0.5, size=(2, B, nx, ny)).astype(np.float32)
    for n, accel, warm in ((1, False, False), (6, False, False), (6, True, False), (5, False, True)):
        prm = sc.tv_params(tv=tv, lam=0.1, n_inner=n, accel=accel, chambolle04=True)
        dual = torch.empty((2, B, nx, ny), device="cuda")
        th, _, its, _ = sc.sci_tv_denoise(ctx, dev(x), prm, dual_init=dev(p0) if warm else None, dual_out=dual)
        ref, pref = orc.tv_denoise(x, f32(0.1), n, tv, accel=accel, chambolle04=True,
                                   p_init=p0 if warm else None, return_dual=True)
        e = rel_l2(host(th), ref)
        ep = np.abs(host(dual) - pref).max()
        say(f"chambolle04 {tv} B={B} {nx}x{ny} N={n} accel={accel} warm={warm}: rel-L2 {e:.2e}, dual {ep:.2e}")
        assert e <= REL_TOL and ep <= 1e-4
    with pytest.raises(RuntimeError):  # 16-bit storage: streaming only
        sc.sci_tv_denoise(ctx, dev(x), sc.tv_params(tv=tv, n_inner=3, chambolle04=True, dual_dtype="bf16",
                                                    schedule="fused"))


@pytest.mark.parametrize("dt,bound", [("bf16", 2e-2), ("f16", 3e-3)])
@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_chambolle04_16bit_duals(sc, ctx, tv, dt, bound):
    """The Chambolle-2004 step with 16-bit dual storage (streaming schedule,
    which the automatic schedule picks for it): float32 arithmetic, rounding
    at every store, so the error against the FP64 oracle is bounded as for
    the projection step (4 lambda u per iteration); cold and warm, with and
    without momentum; the automatic and streaming schedules agree bit for
    bit."""
    r = np.random.default_rng(31)
    B, nx, ny = 5, 50, 130
    x = r.uniform(size=(B, nx, ny)).astype(np.float32)
    ddt = sc.DUAL_TORCH[sc.DUAL[dt]]
    p0 = dev(r.uniform(-0.5, 0.5, size=(2, B, nx, ny)).astype(np.float32), ddt)
    u = 2.0 ** -8 if dt == "bf16" else 2.0 ** -11
    for accel, warm in ((False, False), (True, False), (False, True)):
        outs = []
        for schedule in ("auto", "stream"):
            prm = sc.tv_params(tv=tv, lam=0.1, n_inner=10, accel=accel, chambolle04=True, dual_dtype=dt,
                               schedule=schedule)
            th, _, its, _ = sc.sci_tv_denoise(ctx, dev(x), prm, dual_init=p0 if warm else None)
            assert its == 10
            outs.append(host(th))
        np.testing.assert_array_equal(outs[0], outs[1])
        ref = orc.tv_denoise(x, f32(0.1), 10, tv, accel=accel, chambolle04=True,
                             p_init=host(p0) if warm else None)
        e = rel_l2(outs[0], ref)
        amax = np.abs(outs[0] - ref).max()
        say(f"chambolle04 {tv} {dt} accel={accel} warm={warm}: rel-L2 {e:.2e}, max-abs {amax:.2e}")
        assert e <= bound
        assert amax <= 10 * 4 * 0.1 * u


@pytest.mark.parametrize("dt,bound", [("bf16", 5e-3), ("f16", 1e-3)])
def test_chambolle04_16bit_gap_solve(sc, ctx, dt, bound):
    """GAP-ITV2D with the Chambolle-2004 step, the warm dual kept in 16 bits
    between outer iterations, against the FP64 oracle."""
    pr = synth.make_problem(60, 90, 8, seed=61, sigma=0.01)
    Y = orc.measurement(pr.masks, pr.truth, pr.noise)
    x, _ = run_solver(sc, ctx, "gap", Y, pr.masks, outer_iters=4, tv="itv2d", lam=0.1, n_inner=7, warm_dual=True,
                      chambolle04=True, dual_dtype=dt)
    xr, _ = orc.gap_tv(Y, pr.masks, f32(0.1), 4, 7, tv="itv2d", warm_dual=True, chambolle04=True)
    e = rel_l2(x, xr)
    say(f"GAP-ITV2D chambolle04 {dt} 4 x 7 warm: rel-L2 {e:.2e}")
    assert e <= bound


@pytest.mark.parametrize("tv", ["atv", "itv2d"])
@pytest.mark.parametrize("B,nx,ny", [(1, 1, 1), (2, 5, 3), (3, 130, 64), (2, 300, 130), (1, 97, 214)])
def test_chambolle04_fused_bitwise_equals_streaming(sc, ctx, tv, B, nx, ny):
    """Chambolle-2004 step on the row-pipelined shapes against its streaming
    pass: every row shape, one pass and several, cold and warm starts,
    momentum off and on, final dual returned: identical bits."""
    r = np.random.default_rng(B * 9 + nx + ny)
    x = dev(r.uniform(size=(B, nx, ny)).astype(np.float32))
    p0 = dev(r.uniform(-0.5, 0.5, size=(2, B, nx, ny)).astype(np.float32))
    for n, passes, accel, warm in ((1, 1, False, False), (6, 1, False, False), (6, 2, False, True),
                                   (10, 1, True, False), (13, 2, False, True)):
        init = p0 if warm else None
        prm = sc.tv_params(tv=tv, lam=0.1, n_inner=n, accel=accel, chambolle04=True, schedule="stream")
        dref = torch.empty((2, B, nx, ny), device="cuda")
        tref, _, _, _ = sc.sci_tv_denoise(ctx, x, prm, dual_init=init, dual_out=dref)
        tref, dref = host(tref), host(dref)
        for k in [0] + row_shapes(sc):
            prm = sc.tv_params(tv=tv, lam=0.1, n_inner=n, accel=accel, chambolle04=True, schedule="fused",
                               tile_shape=k, tile_passes=passes)
            d = torch.empty((2, B, nx, ny), device="cuda")
            th, _, its, _ = sc.sci_tv_denoise(ctx, x, prm, dual_init=init, dual_out=d)
            msg = f"shape {k} N={n} passes={passes} accel={accel} warm={warm}"
            assert its == n, msg
            np.testing.assert_array_equal(host(th), tref, err_msg="theta " + msg)
            np.testing.assert_array_equal(host(d), dref, err_msg="dual " + msg)


@pytest.mark.parametrize("B,nx,ny", [(1, 1, 1), (3, 2, 5), (10, 130, 150), (16, 40, 70), (24, 64, 64), (29, 9, 130)])
def test_chambolle04_vtv_fused_bitwise_equals_streaming(sc, ctx, B, nx, ny):
    """VTV with the Chambolle-2004 step: the fused (row-pipelined) kernel
    against the streaming pass, one pass and several, cold and warm starts:
    identical bits."""
    r = np.random.default_rng(B * 19 + nx + ny)
    x = dev(r.uniform(size=(B, nx, ny)).astype(np.float32))
    p0 = dev(r.uniform(-0.3, 0.3, size=(2, B, nx, ny)).astype(np.float32))
    for n, accel, warm in ((1, False, False), (5, False, False), (10, False, True), (7, True, False)):
        init = p0 if warm else None
        outs = []
        for schedule in ("stream", "fused"):
            prm = sc.tv_params(tv="vtv", lam=0.1, n_inner=n, accel=accel, chambolle04=True, schedule=schedule)
            d = torch.empty((2, B, nx, ny), device="cuda")
            th, _, its, _ = sc.sci_tv_denoise(ctx, x, prm, dual_init=init, dual_out=d)
            assert its == n
            outs.append((host(th), host(d)))
        msg = f"VTV Chambolle-2004 B={B} {nx}x{ny} N={n} accel={accel} warm={warm}"
        np.testing.assert_array_equal(outs[1][0], outs[0][0], err_msg="theta " + msg)
        np.testing.assert_array_equal(outs[1][1], outs[0][1], err_msg="dual " + msg)


@pytest.mark.parametrize("solver", ["gap", "admm"])
def test_chambolle04_fused_solvers_bitwise(sc, ctx, solver):
    """GAP / ADMM solves with the Chambolle-2004 step, with and without the
    warm dual: the fused schedule gives the bits of the streaming one."""
    pr = synth.make_problem(150, 90, 6, seed=41, sigma=0.01)
    Y = orc.measurement(pr.masks, pr.truth, pr.noise)
    for warm in (False, True):
        kw = dict(outer_iters=4, rho=0.01, tv="itv2d", lam=0.1, n_inner=7, warm_dual=warm, chambolle04=True,
                  accel=False)
        xs, ts = run_solver(sc, ctx, solver, Y, pr.masks, schedule="stream", **kw)
        xf, tf = run_solver(sc, ctx, solver, Y, pr.masks, schedule="fused", **kw)
        np.testing.assert_array_equal(xf, xs, err_msg=f"{solver} warm={warm}")
        np.testing.assert_array_equal(tf, ts, err_msg=f"{solver} warm={warm}")


@pytest.mark.parametrize("solver", ["gap", "admm"])
@pytest.mark.parametrize("B", [10, 24])
def test_vtv_multipass_fused_solvers_bitwise(sc, ctx, solver, B):
    """GAP / ADMM with VTV and 10 inner iterations per call, which the fused
    schedule runs as two passes handing the duals over as one record per
    voxel (B = 10: 2 frames per wavefront, B = 24: 3), with and without the
    warm dual: the bits of the streaming schedule, and the oracle's result
    within the usual tolerance."""
    pr = synth.make_problem(70, 90, B, seed=43 + B, sigma=0.01)
    Y = orc.measurement(pr.masks, pr.truth, pr.noise)
    for warm in (False, True):
        kw = dict(outer_iters=3, rho=0.01, tv="vtv", lam=0.1, n_inner=10, warm_dual=warm)
        xs, ts = run_solver(sc, ctx, solver, Y, pr.masks, schedule="stream", **kw)
        xf, tf = run_solver(sc, ctx, solver, Y, pr.masks, schedule="fused", **kw)
        np.testing.assert_array_equal(xf, xs, err_msg=f"{solver} B={B} warm={warm}")
        np.testing.assert_array_equal(tf, ts, err_msg=f"{solver} B={B} warm={warm}")
        if solver == "gap":
            xr, _ = orc.gap_tv(Y, pr.masks, f32(0.1), 3, 10, tv="vtv", warm_dual=warm)
        else:
            xr, _ = orc.admm_tv(Y, pr.masks, f32(0.1), f32(0.01), 3, 10, tv="vtv", warm_dual=warm)
        e = rel_l2(xf, xr)
        say(f"{solver}-VTV B={B} 3 x 10 warm={warm}, fused (two passes, records) vs oracle: rel-L2 {e:.2e}")
        assert e <= REL_TOL


@pytest.mark.parametrize("dt,bound", [("f32", REL_TOL), ("bf16", 5e-5), ("f16", 5e-6)])
@pytest.mark.parametrize("solver", ["gap", "admm"])
def test_vtv_multipass_graph_replays(sc, ctx, solver, dt, bound):
    """The same two-pass VTV solves (B = 24, records between the passes in the
    storage type) captured in a HIP graph: every replay, with eager solves
    between them, gives the bits of the eager solve; the result is within
    about ten times the measured error of the oracle (rounding to 16 bits at
    each pass boundary: 3-4e-6 bf16, 4-6e-7 fp16)."""
    B = 24
    pr = synth.make_problem(66, 75, B, seed=77, sigma=0.01)
    Y = orc.measurement(pr.masks, pr.truth, pr.noise)
    for warm in (False, True):
        kw = dict(outer_iters=3, rho=0.01, tv="vtv", lam=0.1, n_inner=10, warm_dual=warm, dual_dtype=dt,
                  schedule="fused")
        xe, te = run_solver(sc, ctx, solver, Y, pr.masks, **kw)
        for rep in range(3):
            xg, tg = run_solver(sc, ctx, solver, Y, pr.masks, use_graph=True, **kw)
            np.testing.assert_array_equal(xg, xe, err_msg=f"{solver} {dt} warm={warm} replay {rep}")
            np.testing.assert_array_equal(tg, te, err_msg=f"{solver} {dt} warm={warm} replay {rep}")
            xe2, _ = run_solver(sc, ctx, solver, Y, pr.masks, **kw)  # eager work between replays
            np.testing.assert_array_equal(xe2, xe)
        if solver == "gap":
            xr, _ = orc.gap_tv(Y, pr.masks, f32(0.1), 3, 10, tv="vtv", warm_dual=warm)
        else:
            xr, _ = orc.admm_tv(Y, pr.masks, f32(0.1), f32(0.01), 3, 10, tv="vtv", warm_dual=warm)
        e = rel_l2(xe, xr)
        say(f"{solver}-VTV B={B} {dt} 3 x 10 warm={warm}, graph = eager; vs oracle rel-L2 {e:.2e}")
        assert e <= bound


@pytest.mark.parametrize("B,nx,ny", [(1, 1, 1), (1, 2, 2), (2, 5, 3), (3, 17, 63), (4, 130, 64), (24, 16, 64)])
def test_clip_matches_oracle(sc, ctx, B, nx, ny):
    """ATV-Clip: per-direction iterative clipping, threshold 2 lambda."""
    r = np.random.default_rng(B * 3 + nx * 5 + ny)
    x = r.uniform(size=(B, nx, ny)).astype(np.float32)
    w0 = r.uniform(-0.1, 0.1, size=(2, B, nx, ny)).astype(np.float32)
    for n, alpha, warm in ((1, 0.0, False), (8, 0.0, False), (8, 3.0, False), (5, 4.5, True)):
        prm = sc.tv_params(tv="atv", lam=0.05, n_inner=n, clip=True, clip_alpha=alpha)
        dual = torch.empty((2, B, nx, ny), device="cuda")
        th, _, _, _ = sc.sci_tv_denoise(ctx, dev(x), prm, dual_init=dev(w0) if warm else None, dual_out=dual)
        ref, wref = orc.clip_denoise(x, f32(0.05), n, f32(alpha) if alpha else 4.0, w_init=w0 if warm else None,
                                     return_dual=True)
        e = rel_l2(host(th), ref)
        ew = np.abs(host(dual) - wref).max()
        say(f"clip B={B} {nx}x{ny} N={n} alpha={alpha} warm={warm}: rel-L2 {e:.2e}, dual {ew:.2e}")
        assert e <= REL_TOL and ew <= 1e-6
    for bad in (dict(tv="itv2d"), dict(tv="atv", dual_dtype="bf16", schedule="fused"),
                dict(tv="atv", gap_tol=1e-3, n_inner_max=10)):
        with pytest.raises(RuntimeError):
            sc.sci_tv_denoise(ctx, dev(x), sc.tv_params(lam=0.05, n_inner=3, clip=True, **bad))


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_clip_16bit_duals(sc, ctx, dt):
    """ATV-Clip with 16-bit dual storage (streaming schedule, which the
    automatic schedule picks for it), cold and warm: the automatic and
    streaming schedules agree bit for bit; against the FP64 oracle the
    error stays within the rounding of the stores (each |w| <= 2 lambda is
    stored with relative error u, and theta = x - D^T w takes four of them:
    at most n * 8 lambda u after n non-expansive iterations), and the
    returned dual is the oracle's to within one rounding per iteration."""
    r = np.random.default_rng(41)
    B, nx, ny, lam, n = 3, 50, 130, 0.05, 8
    x = r.uniform(size=(B, nx, ny)).astype(np.float32)
    ddt = sc.DUAL_TORCH[sc.DUAL[dt]]
    w0 = dev(r.uniform(-0.1, 0.1, size=(2, B, nx, ny)).astype(np.float32), ddt)
    u = 2.0 ** -8 if dt == "bf16" else 2.0 ** -11
    for warm in (False, True):
        outs, duals = [], []
        for schedule in ("auto", "stream"):
            prm = sc.tv_params(tv="atv", lam=lam, n_inner=n, clip=True, dual_dtype=dt, schedule=schedule)
            dual = torch.empty((2, B, nx, ny), device="cuda", dtype=ddt)
            th, _, _, _ = sc.sci_tv_denoise(ctx, dev(x), prm, dual_init=w0 if warm else None, dual_out=dual)
            outs.append(host(th))
            duals.append(host(dual))
        np.testing.assert_array_equal(outs[0], outs[1])
        np.testing.assert_array_equal(duals[0], duals[1])
        ref, wref = orc.clip_denoise(x, f32(lam), n, 4.0, w_init=host(w0) if warm else None, return_dual=True)
        amax = np.abs(outs[0] - ref).max()
        ew = np.abs(duals[0] - wref).max()
        say(f"clip {dt} warm={warm}: rel-L2 {rel_l2(outs[0], ref):.2e}, max-abs {amax:.2e} "
            f"(bound {n * 8 * lam * u:.2e}), dual {ew:.2e}")
        assert amax <= n * 8 * lam * u
        assert ew <= n * 2 * lam * u


@pytest.mark.parametrize("B,nx,ny", [(1, 1, 1), (2, 5, 3), (3, 130, 64), (2, 300, 130), (1, 97, 214)])
def test_clip_fused_bitwise_equals_streaming(sc, ctx, B, nx, ny):
    """ATV-Clip on the row-pipelined kernel against one pass per iteration:
    every row shape, one pass and several, cold and warm starts, final duals
    returned: identical bits."""
    r = np.random.default_rng(B * 17 + nx + ny)
    x = dev(r.uniform(size=(B, nx, ny)).astype(np.float32))
    w0 = dev(r.uniform(-0.1, 0.1, size=(2, B, nx, ny)).astype(np.float32))
    for n, passes, alpha, warm in ((1, 0, 0.0, False), (4, 0, 3.0, True), (10, 0, 0.0, False), (13, 2, 4.5, True),
                                   (25, 0, 0.0, False)):
        init = w0 if warm else None
        prm = sc.tv_params(tv="atv", lam=0.05, n_inner=n, clip=True, clip_alpha=alpha, schedule="stream")
        dref = torch.empty((2, B, nx, ny), device="cuda")
        tref, _, _, _ = sc.sci_tv_denoise(ctx, x, prm, dual_init=init, dual_out=dref)
        tref, dref = host(tref), host(dref)
        for k in [0] + row_shapes(sc):
            prm = sc.tv_params(tv="atv", lam=0.05, n_inner=n, clip=True, clip_alpha=alpha, schedule="fused",
                               tile_shape=k, tile_passes=passes)
            d = torch.empty((2, B, nx, ny), device="cuda")
            th, _, its, _ = sc.sci_tv_denoise(ctx, x, prm, dual_init=init, dual_out=d)
            msg = f"shape {k} N={n} passes={passes} alpha={alpha} warm={warm}"
            assert its == n, msg
            np.testing.assert_array_equal(host(th), tref, err_msg="theta " + msg)
            np.testing.assert_array_equal(host(d), dref, err_msg="dual " + msg)


@pytest.mark.parametrize("solver", ["gap", "admm"])
def test_clip_fused_solvers_bitwise(sc, ctx, solver):
    """GAP / ADMM with ATV-Clip (ADMM takes u = s - theta from the kernel), with
    and without the warm dual: the fused schedule gives the streaming bits."""
    pr = synth.make_problem(150, 90, 6, seed=51, sigma=0.01)
    Y = orc.measurement(pr.masks, pr.truth, pr.noise)
    for warm in (False, True):
        kw = dict(outer_iters=4, rho=0.05, tv="atv", lam=0.05, n_inner=6, clip=True, warm_dual=warm)
        xs, ts = run_solver(sc, ctx, solver, Y, pr.masks, schedule="stream", **kw)
        xf, tf = run_solver(sc, ctx, solver, Y, pr.masks, schedule="fused", **kw)
        np.testing.assert_array_equal(xf, xs, err_msg=f"{solver} warm={warm}")
        np.testing.assert_array_equal(tf, ts, err_msg=f"{solver} warm={warm}")


@pytest.mark.parametrize("solver", ["gap", "admm"])
def test_clip_outer_matches_oracle(sc, ctx, solver):
    pr = synth.make_problem(96, 130, 8, seed=19, sigma=0.01)
    Y = orc.measurement(pr.masks, pr.truth, pr.noise)
    cold = None
    for warm in (False, True):
        x, th = run_solver(sc, ctx, solver, Y, pr.masks, outer_iters=10, rho=0.05, tv="atv", lam=0.05,
                           n_inner=6, clip=True, warm_dual=warm)
        cold = x if not warm else cold
        if solver == "gap":
            xr, thr = orc.gap_tv(Y, pr.masks, f32(0.05), 10, 6, tv="atv", clip=True, warm_dual=warm)
        else:
            xr, thr = orc.admm_tv(Y, pr.masks, f32(0.05), f32(0.05), 10, 6, tv="atv", clip=True, warm_dual=warm)
        e = rel_l2(x, xr)
        say(f"{solver}-ATV-Clip warm={warm}: rel-L2 {e:.2e}, PSNR {orc.psnr(xr, pr.truth):.2f}")
        assert e <= REL_TOL and rel_l2(th, thr) <= REL_TOL
    # the captured graph replays the same arithmetic
    Yd, Cd = dev(Y), dev(pr.masks)
    fn = sc.sci_gap_tv if solver == "gap" else sc.sci_admm_tv
    prm = sc.solver_params(outer_iters=10, rho=0.05, tv="atv", lam=0.05, n_inner=6, clip=True, use_graph=True)
    for _ in range(2):
        xg, _ = fn(ctx, Yd, Cd, prm)
        np.testing.assert_array_equal(host(xg), cold)


@pytest.mark.parametrize("dt,bound", [("bf16", 2e-2), ("f16", 3e-3)])
@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_denoise_16bit_duals(sc, ctx, tv, dt, bound):
    """16-bit dual storage: float32 arithmetic, rounding at every store. The
    error against the FP64 oracle is bounded by the per-store rounding
    (4 lambda u per iteration for u = 2^-8 (bf16) / 2^-11 (f16))."""
    x = np.random.default_rng(9).uniform(size=(4, 50, 130)).astype(np.float32)
    prm = sc.tv_params(tv=tv, lam=0.1, n_inner=10, dual_dtype=dt)
    th, _, _, _ = sc.sci_tv_denoise(ctx, dev(x), prm)
    ref = orc.tv_denoise(x, f32(0.1), 10, tv)
    e = rel_l2(host(th), ref)
    amax = np.abs(host(th) - ref).max()
    u = 2.0 ** -8 if dt == "bf16" else 2.0 ** -11
    say(f"{tv} {dt} duals: rel-L2 {e:.2e}, max-abs {amax:.2e} (per-step bound {4 * 0.1 * u:.2e})")
    assert e <= bound
    assert amax <= 10 * 4 * 0.1 * u


@pytest.mark.parametrize("dt,bound", [("bf16", 2e-2), ("f16", 3e-3)])
@pytest.mark.parametrize("B,maxpass", [(8, 10), (16, 10), (24, 7), (32, 4)])
def test_vtv_fused_16bit_duals_between_passes(sc, ctx, B, maxpass, dt, bound):
    """VTV on the fused schedule with 16-bit dual storage: a call longer than
    one pass (at most 10 / 10 / 7 / 4 iterations for B <= 8 / 16 / 24 / 32)
    stores the dual between passes in 16 bits and keeps it in float32
    registers inside a pass. Against the FP64 oracle within the 16-bit bound,
    cold and from a 16-bit starting dual, with the returned dual checked
    through the duality gap it certifies; beside it the streaming schedule,
    which rounds after every iteration."""
    r = np.random.default_rng(B)
    nx, ny = 37, 70
    x = r.uniform(size=(B, nx, ny)).astype(np.float32)
    n = 2 * maxpass + 1  # three passes
    ddt = sc.DUAL_TORCH[sc.DUAL[dt]]
    p0 = orc.project_dual(0.3 * r.normal(size=(2, B, nx, ny)), "vtv")
    p0_16 = dev(p0.astype(np.float32), ddt)
    for init in (None, p0_16):
        errs = {}
        for schedule in ("fused", "stream"):
            prm = sc.tv_params(tv="vtv", lam=0.1, n_inner=n, schedule=schedule, dual_dtype=dt)
            dual = torch.empty((2, B, nx, ny), device="cuda", dtype=ddt)
            th, gap, its, _ = sc.sci_tv_denoise(ctx, dev(x), prm, dual_init=init, dual_out=dual, want_gap=True)
            assert its == n
            ref = orc.tv_denoise(x, f32(0.1), n, "vtv", p_init=None if init is None else host(init))
            errs[schedule] = rel_l2(host(th), ref)
            # the returned dual is feasible and certifies theta through the FP64 gap
            g, prim = orc.dual_gap(x, host(dual), f32(0.1), "vtv")
            assert np.isfinite(gap) and abs(gap - g / prim) <= 1e-3 * max(g / prim, 1e-6) + 1e-6
        say(f"vtv B={B} {dt} N={n} ({'warm' if init is not None else 'cold'}): rel-L2 fused {errs['fused']:.2e}, "
            f"streaming {errs['stream']:.2e}")
        assert errs["fused"] <= bound and errs["stream"] <= bound


@pytest.mark.parametrize("dt", ["bf16", "f16"])
@pytest.mark.parametrize("B,m", [(16, 8), (24, 7), (32, 4)])
def test_vtv_16bit_records_equal_chained_calls(sc, ctx, B, m, dt):
    """A fused VTV call of three passes with 16-bit dual storage hands the
    dual from pass to pass as one record per voxel, rounded to the storage
    type. Without acceleration each pass depends only on the dual it starts
    from, so the call equals three calls of one pass each chained through a
    16-bit dual_out / dual_init, bit for bit (theta and the returned dual),
    cold and from a starting dual."""
    r = np.random.default_rng(900 + B)
    nx, ny = 37, 70
    x = dev(r.uniform(size=(B, nx, ny)).astype(np.float32))
    ddt = sc.DUAL_TORCH[sc.DUAL[dt]]
    p0 = dev(orc.project_dual(0.3 * r.normal(size=(2, B, nx, ny)), "vtv").astype(np.float32), ddt)
    for init in (None, p0):
        prm = sc.tv_params(tv="vtv", lam=0.1, n_inner=3 * m, accel=False, dual_dtype=dt)
        d_one = torch.empty((2, B, nx, ny), device="cuda", dtype=ddt)
        th_one, _, its, _ = sc.sci_tv_denoise(ctx, x, prm, dual_init=init, dual_out=d_one)
        assert its == 3 * m
        prm1 = sc.tv_params(tv="vtv", lam=0.1, n_inner=m, accel=False, dual_dtype=dt)
        d = init
        for _ in range(3):
            d_next = torch.empty((2, B, nx, ny), device="cuda", dtype=ddt)
            th, _, its, _ = sc.sci_tv_denoise(ctx, x, prm1, dual_init=d, dual_out=d_next)
            assert its == m
            d = d_next
        np.testing.assert_array_equal(host(th_one), host(th))
        np.testing.assert_array_equal(d_one.view(torch.int16).cpu().numpy(), d.view(torch.int16).cpu().numpy())


# ---------------------------------------------------------------------------
# GAP / ADMM.
# ---------------------------------------------------------------------------

def run_solver(sc, ctx, solver, Y, C, **kw):
    prm = sc.solver_params(**kw)
    fn = sc.sci_gap_tv if solver == "gap" else sc.sci_admm_tv
    th = torch.empty(C.shape, device="cuda")
    x, _ = fn(ctx, dev(Y), dev(C), prm, Theta_out=th)
    return host(x), host(th)


def oracle_solver(solver, Y, C, lam, rho, T, N, tv):
    if solver == "gap":
        return orc.gap_tv(Y, C, f32(lam), T, N, tv=tv)
    return orc.admm_tv(Y, C, f32(lam), f32(rho), T, N, tv=tv)


def test_gap_atv_256x8(sc, ctx):
    cfg = synth.CONFIGS["gap_atv_256x8"]
    pr = synth.problem_from_config("gap_atv_256x8")
    Y = orc.measurement(pr.masks, pr.truth, pr.noise)
    x, th = run_solver(sc, ctx, "gap", Y, pr.masks, outer_iters=cfg["T"], tv="atv", lam=cfg["lam"],
                       n_inner=cfg["N"])
    xr, thr = orc.gap_tv(Y, pr.masks, f32(cfg["lam"]), cfg["T"], cfg["N"], tv="atv")
    e, dp = rel_l2(x, xr), abs(orc.psnr(x, pr.truth) - orc.psnr(xr, pr.truth))
    say(f"GAP-ATV 256x256x8 50x5: rel-L2 {e:.2e}, dPSNR {dp:.2e} dB, PSNR {orc.psnr(xr, pr.truth):.2f}")
    assert e <= REL_TOL and dp <= PSNR_TOL
    assert rel_l2(th, thr) <= REL_TOL


@pytest.fixture(scope="module")
def six_problem():
    pr = synth.problem_from_config("six_256x8")
    return pr, orc.measurement(pr.masks, pr.truth, pr.noise), {}


@pytest.mark.parametrize("schedule", ["auto", "stream"])
@pytest.mark.parametrize("solver", ["gap", "admm"])
@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_six_variants_256x8(sc, ctx, six_problem, solver, tv, schedule):
    cfg = synth.CONFIGS["six_256x8"]
    pr, Y, cache = six_problem
    x, th = run_solver(sc, ctx, solver, Y, pr.masks, outer_iters=cfg["T"], rho=cfg["rho"], tv=tv,
                       lam=cfg["lam"], n_inner=cfg["N"], schedule=schedule)
    if (solver, tv) not in cache:
        cache[(solver, tv)] = oracle_solver(solver, Y, pr.masks, cfg["lam"], cfg["rho"], cfg["T"], cfg["N"], tv)
    xr, thr = cache[(solver, tv)]
    e, dp = rel_l2(x, xr), abs(orc.psnr(x, pr.truth) - orc.psnr(xr, pr.truth))
    say(f"{solver}-{tv}/{schedule} 256x256x8 100x10: rel-L2 {e:.2e}, dPSNR {dp:.2e} dB, "
        f"oracle PSNR {orc.psnr(xr, pr.truth):.2f}")
    assert e <= REL_TOL and dp <= PSNR_TOL
    assert rel_l2(th, thr) <= REL_TOL


@pytest.mark.parametrize("solver", ["gap", "admm"])
def test_ragged_small_solves(sc, ctx, solver):
    for (B, nx, ny), tv in (((3, 37, 101), "atv"), ((5, 64, 63), "itv2d"), ((10, 29, 130), "vtv"), ((1, 1, 1), "atv")):
        pr = synth.make_problem(nx, ny, B, seed=nx + ny, sigma=0.01, radius=(2.0, 8.0))
        Y = orc.measurement(pr.masks, pr.truth, pr.noise)
        x, th = run_solver(sc, ctx, solver, Y, pr.masks, outer_iters=7, rho=0.05, tv=tv, lam=0.1, n_inner=4)
        xr, thr = oracle_solver(solver, Y, pr.masks, 0.1, 0.05, 7, 4, tv)
        assert rel_l2(x, xr) <= REL_TOL, (B, nx, ny, tv)
        assert rel_l2(th, thr) <= REL_TOL, (B, nx, ny, tv)


@pytest.mark.parametrize("solver", ["gap", "admm"])
@pytest.mark.parametrize("tv,cham", [("atv", False), ("itv2d", False), ("vtv", False), ("itv2d", True),
                                     ("vtv", True)])
def test_warm_dual_and_chambolle04_outer_match_oracle(sc, ctx, solver, tv, cham):
    """Outer loops with the dual carried across outer iterations (and the
    Chambolle-2004 step) against the oracle's drivers."""
    pr = synth.make_problem(70, 90, 6, seed=17, sigma=0.01, radius=(3.0, 12.0))
    Y = orc.measurement(pr.masks, pr.truth, pr.noise)
    for warm in (True, False) if cham else (True,):
        x, th = run_solver(sc, ctx, solver, Y, pr.masks, outer_iters=9, rho=0.05, tv=tv, lam=0.1, n_inner=4,
                           warm_dual=warm, chambolle04=cham)
        fn = orc.gap_tv if solver == "gap" else (lambda *a, **k: orc.admm_tv(a[0], a[1], a[2], f32(0.05), *a[3:], **k))
        xr, thr = fn(Y, pr.masks, f32(0.1), 9, 4, tv=tv, warm_dual=warm, chambolle04=cham)
        e = rel_l2(x, xr)
        say(f"{solver} {tv} warm={warm} chambolle04={cham}: rel-L2 {e:.2e}")
        assert e <= REL_TOL and rel_l2(th, thr) <= REL_TOL


@pytest.mark.parametrize("solver", ["gap", "admm"])
@pytest.mark.parametrize("tv", ["atv", "vtv"])
def test_warm_dual_schedules_agree(sc, ctx, solver, tv):
    """Keeping the dual across outer iterations: the fused and streaming
    schedules agree bit for bit, and both differ from the cold start."""
    pr = synth.make_problem(130, 120, 6, seed=16, sigma=0.01)
    Y = orc.measurement(pr.masks, pr.truth, pr.noise)
    outs = {}
    for schedule in ("stream", "auto"):
        outs[schedule] = run_solver(sc, ctx, solver, Y, pr.masks, outer_iters=8, rho=0.01, tv=tv, n_inner=5,
                                    warm_dual=True, schedule=schedule)
    np.testing.assert_array_equal(outs["stream"][0], outs["auto"][0])
    cold = run_solver(sc, ctx, solver, Y, pr.masks, outer_iters=8, rho=0.01, tv=tv, n_inner=5)
    assert np.abs(cold[0] - outs["auto"][0]).max() > 1e-6


@pytest.mark.parametrize("solver", ["gap", "admm"])
@pytest.mark.parametrize("kind", ["binary", "graded", "binary_b40"])
def test_mask_kinds_match_oracle(sc, ctx, solver, kind):
    """Binary masks (B <= 32) take the packed-bit projection, graded masks
    (entries in (0, 1]) and more than 32 frames the float path; all match the
    oracle."""
    B = 40 if kind == "binary_b40" else 6
    pr = synth.make_problem(70, 66, B, seed=21, sigma=0.01)
    C = pr.masks
    if kind == "graded":
        C = (C * np.random.default_rng(22).uniform(0.2, 1.0, size=C.shape)).astype(np.float32)
    Y = orc.measurement(C, pr.truth, pr.noise)
    tv = "atv" if B > 32 else "vtv"
    x, th = run_solver(sc, ctx, solver, Y, C, outer_iters=6, rho=0.05, tv=tv, lam=0.1, n_inner=5)
    xr, thr = oracle_solver(solver, Y, C, 0.1, 0.05, 6, 5, tv)
    e = rel_l2(x, xr)
    say(f"{solver} {kind} masks B={B}: rel-L2 {e:.2e}")
    assert e <= REL_TOL and rel_l2(th, thr) <= REL_TOL


@pytest.mark.parametrize("solver", ["gap", "admm"])
def test_graph_replay_matches_eager(sc, ctx, solver):
    pr = synth.make_problem(96, 80, 8, seed=12, sigma=0.01)
    Y = orc.measurement(pr.masks, pr.truth, pr.noise)
    x0, t0 = run_solver(sc, ctx, solver, Y, pr.masks, outer_iters=6, rho=0.01, tv="itv2d", n_inner=5)
    Yd, Cd = dev(Y), dev(pr.masks)
    prm = sc.solver_params(outer_iters=6, rho=0.01, tv="itv2d", n_inner=5, use_graph=True)
    fn = sc.sci_gap_tv if solver == "gap" else sc.sci_admm_tv
    xg = torch.empty(Cd.shape, device="cuda")
    tg = torch.empty(Cd.shape, device="cuda")
    for rep in range(3):
        xg.fill_(float("nan"))
        fn(ctx, Yd, Cd, prm, X_out=xg, Theta_out=tg)
        _ = torch.ones(1000, device="cuda").sum().item()  # unrelated eager work between replays
        np.testing.assert_array_equal(host(xg), x0)
        np.testing.assert_array_equal(host(tg), t0)


def test_graph_replay_after_workspace_growth(sc, ctx):
    """A cached graph holds workspace addresses: a larger solve in between
    grows (frees and reallocates) the workspace, and the next graph call of
    the small problem must still match the eager result. A context of its own
    starts with an empty workspace, so the larger solve does grow it."""
    own = sc.Context(0)
    try:
        _graph_after_growth(sc, own.handle, ctx)
    finally:
        own.close()


def _graph_after_growth(sc, g, ctx):
    small = synth.make_problem(96, 80, 8, seed=13, sigma=0.01)
    big = synth.make_problem(256, 192, 12, seed=14, sigma=0.01)
    Ys = orc.measurement(small.masks, small.truth, small.noise)
    Yb = orc.measurement(big.masks, big.truth, big.noise)
    kw = dict(outer_iters=4, tv="itv2d", lam=0.1, n_inner=5)
    prm = sc.solver_params(use_graph=True, **kw)
    Yd, Cd = dev(Ys), dev(small.masks)
    xg = torch.empty(Cd.shape, device="cuda")
    sc.sci_gap_tv(g, Yd, Cd, prm, X_out=xg)  # captured with the small workspace
    first = host(xg)
    xb, _ = sc.sci_gap_tv(g, dev(Yb), dev(big.masks), sc.solver_params(**kw))  # grows every slot it uses
    xg.fill_(float("nan"))
    sc.sci_gap_tv(g, Yd, Cd, prm, X_out=xg)
    x0, _ = run_solver(sc, ctx, "gap", Ys, small.masks, **kw)
    np.testing.assert_array_equal(first, x0)
    np.testing.assert_array_equal(host(xg), x0)
    assert np.isfinite(host(xb)).all()


@pytest.mark.parametrize("solver", ["gap", "admm"])
@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_constant_frames_fixed_point(sc, ctx, solver, tv):
    B, nx, ny = 4, 40, 70
    truth = np.broadcast_to(np.array([0.2, 0.5, 0.9, 0.1], np.float32)[:, None, None], (B, nx, ny)).copy()
    C = synth.masks_bernoulli(np.random.default_rng(13), nx, ny, B)
    Y = orc.measurement(C, truth)
    prm = sc.solver_params(outer_iters=5, rho=0.01, tv=tv, n_inner=5)
    fn = sc.sci_gap_tv if solver == "gap" else sc.sci_admm_tv
    x, _ = fn(ctx, dev(Y), dev(C), prm, X_init=dev(truth))
    assert np.abs(host(x) - truth).max() < 1e-6


def test_gap_iterates_satisfy_measurement(sc, ctx):
    pr = synth.make_problem(128, 96, 8, seed=14)
    Y = orc.measurement(pr.masks, pr.truth)
    S = (pr.masks.astype(np.float64) ** 2).sum(axis=0)
    for T in (1, 4):
        x, _ = run_solver(sc, ctx, "gap", Y, pr.masks, outer_iters=T, tv="vtv", n_inner=5)
        f = orc.forward(pr.masks, x)
        assert np.abs(f - Y)[S > 0].max() < 1e-5


@pytest.mark.parametrize("B,nx,ny,binary", [(8, 40, 70, True), (24, 33, 35, True), (10, 64, 64, False),
                                             (40, 32, 32, False)])
def test_admm_x_stored_on_last_pass(sc, ctx, B, nx, ny, binary):
    """ADMM stores x only on its last outer pass (the denoiser reads u + x and
    forms the new u itself). x^(T) must still be the whole projection of Eq. (24):
    with rho = 0 it meets Phi x = y wherever a mask is non-zero, whatever X_out
    held before. The cases reach packed bits, an odd pixel count, real-valued
    masks and B > 32."""
    r = np.random.default_rng(16)
    C = synth.masks_bernoulli(r, nx, ny, B) if binary else r.uniform(size=(B, nx, ny)).astype(np.float32)
    truth = r.uniform(size=(B, nx, ny)).astype(np.float32)
    Y = orc.measurement(C, truth)
    S = (C.astype(np.float64) ** 2).sum(axis=0)
    prm = sc.solver_params(outer_iters=3, rho=0.0, tv="itv2d", n_inner=5)
    outs = []
    for fill in (float("nan"), 0.0):
        xo = torch.full((B, nx, ny), fill, device="cuda")
        sc.sci_admm_tv(ctx, dev(Y), dev(C), prm, X_out=xo)
        outs.append(host(xo))
    np.testing.assert_array_equal(outs[0], outs[1])
    f = orc.forward(C, outs[0])
    assert np.abs(f - Y)[S > 0].max() <= 1e-6 * B * max(1.0, float(np.abs(Y).max()))


def test_metrics_match_oracle(sc, ctx):
    r = np.random.default_rng(15)
    a = r.uniform(size=(6, 33, 71)).astype(np.float32)
    b = (a + r.normal(scale=0.03, size=a.shape)).astype(np.float32)
    assert abs(sc.sci_psnr(ctx, dev(a), dev(b)) - orc.psnr(a, b)) < 1e-9
    C = synth.masks_bernoulli(r, 33, 71, 6)
    Y = r.uniform(size=(33, 71)).astype(np.float32)
    rs = sc.sci_residual_sq(ctx, dev(C), dev(a), dev(Y))
    assert abs(rs - orc.residual_sq(C, a, Y)) <= 1e-12 * rs


def test_errors_are_reported(sc, ctx):
    x = torch.zeros((2, 8, 8), device="cuda")
    with pytest.raises(sc.SciError) as e:
        sc.sci_tv_denoise(ctx, x, sc.tv_params(lam=-1.0))
    assert e.value.status == sc.SCI_ERR_INVALID_ARG
    with pytest.raises(sc.SciError) as e:
        sc.sci_tv_denoise(ctx, x, sc.tv_params(lam=float("nan")))
    assert e.value.status == sc.SCI_ERR_INVALID_ARG
    with pytest.raises(sc.SciError) as e:
        sc.sci_tv_denoise(ctx, x, sc.tv_params(), Theta_out=x)
    assert e.value.status == sc.SCI_ERR_ALIAS
    C = torch.ones((2, 8, 8), device="cuda")
    Y = torch.zeros((8, 8), device="cuda")
    with pytest.raises(sc.SciError) as e:
        sc.sci_gap_tv(ctx, Y, C, sc.solver_params(outer_iters=-1))
    assert e.value.status == sc.SCI_ERR_INVALID_ARG
    with pytest.raises(sc.SciError) as e:
        sc.sci_gap_tv(ctx, Y, C, sc.solver_params(outer_iters=2), X_out=C)
    assert e.value.status == sc.SCI_ERR_ALIAS
    with pytest.raises(sc.SciError) as e:
        big = torch.zeros((49, 4, 4), device="cuda")
        sc.sci_tv_denoise(ctx, big, sc.tv_params(tv="vtv"))
    assert e.value.status == sc.SCI_ERR_UNSUPPORTED
    with pytest.raises(sc.SciError) as e:
        big = torch.zeros((33, 4, 4), device="cuda")
        sc.sci_tv_denoise(ctx, big, sc.tv_params(tv="vtv", schedule="fused"))
    assert e.value.status == sc.SCI_ERR_UNSUPPORTED


# ---------------------------------------------------------------------------
# The large CACTI-style workload at full size.
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def cacti():
    pr = synth.problem_from_config("cacti_1024x24")
    return pr, orc.measurement(pr.masks, pr.truth, pr.noise)


def test_cacti_full_size_two_outer_iterations(sc, ctx, cacti):
    """Same kernels and launch shapes as the benchmark, at 1024x1024x24,
    for two outer iterations the oracle can afford."""
    pr, Y = cacti
    # tile shape and pass count chosen by the autotuner on the back-projection,
    # as the benchmark does before it times the solve
    C = dev(pr.masks)
    x0 = sc.sci_adjoint(ctx, C, dev(Y))
    best, passes, _ = sc.sci_autotune(ctx, x0, sc.tv_params(tv="itv2d", lam=0.1, n_inner=10))
    del x0
    x, th = run_solver(sc, ctx, "gap", Y, pr.masks, outer_iters=2, tv="itv2d", lam=0.1, n_inner=10)
    xr, thr = orc.gap_tv(Y, pr.masks, f32(0.1), 2, 10, tv="itv2d")
    e = rel_l2(x, xr)
    say(f"GAP-ITV2D 1024x1024x24 T=2 (tuned shape {best}, {passes} pass(es)): rel-L2 {e:.2e}")
    assert e <= REL_TOL and rel_l2(th, thr) <= REL_TOL


def test_cacti_full_solve_properties(sc, ctx, cacti):
    """Full 200 x 10 solve: every GAP iterate lies on {Phi x = Y} where
    sum_k C_k^2 > 0, and the reconstruction beats the back-projection."""
    pr, Y = cacti
    x, _ = run_solver(sc, ctx, "gap", Y, pr.masks, outer_iters=200, tv="itv2d", lam=0.1, n_inner=10,
                      use_graph=True)
    assert np.isfinite(x).all()
    S = (pr.masks.astype(np.float64) ** 2).sum(axis=0)
    f = orc.forward(pr.masks, x)
    assert np.abs(f - Y)[S > 0].max() < 1e-4
    p_x = orc.psnr(x, pr.truth)
    p_0 = orc.psnr(orc.adjoint(pr.masks, Y) / np.maximum(S, 1)[None], pr.truth)
    say(f"GAP-ITV2D 1024x1024x24 200x10: PSNR {p_x:.2f} dB (back-projection {p_0:.2f})")
    assert p_x > p_0 + 5.0


@pytest.mark.parametrize("tv", ["atv", "itv2d"])
@pytest.mark.parametrize("B,nx,ny,masks", [(8, 70, 96, "binary"), (24, 33, 130, "binary"), (6, 45, 61, "graded"),
                                           (40, 21, 100, "binary")])
def test_gap_row_and_tiled_shapes_bitwise(sc, ctx, tv, B, nx, ny, masks):
    """Whole GAP solves with the row-pipelined and with a tiled denoiser
    shape give the same bits (the same per-voxel arithmetic): several
    outer-iteration counts, X_init given or not, Theta_out requested or not,
    eager and graph-launched; packed bits (binary masks, B <= 32) and float
    masks (graded, or B > 32) in the projection."""
    pr = synth.make_problem(nx, ny, B, seed=nx + ny + B, sigma=0.01, radius=(3.0, 15.0))
    C = pr.masks
    if masks == "graded":
        C = (C * np.random.default_rng(B).uniform(0.2, 1.0, size=C.shape)).astype(np.float32)
    Y, Cd = dev(orc.measurement(C, pr.truth, pr.noise)), dev(C)
    shapes = range(1, sc.sci_tile_shape_count() + 1)
    row = next(k for k in shapes if sc.sci_tile_shape_pipelined(k))
    tiled = next(k for k in shapes if not sc.sci_tile_shape_pipelined(k))
    x0 = dev(np.random.default_rng(3).uniform(size=C.shape).astype(np.float32))
    for T in (1, 2, 3, 6):
        for x_init in (None, x0):
            for graph in (False, True):
                outs = []
                for shape in (row, tiled):
                    prm = sc.solver_params(outer_iters=T, tv=tv, lam=0.1, n_inner=7, tile_shape=shape,
                                           tile_passes=1, use_graph=graph)
                    th = torch.empty_like(Cd)
                    x, _ = sc.sci_gap_tv(ctx, Y, Cd, prm, Theta_out=th, X_init=x_init)
                    x2, _ = sc.sci_gap_tv(ctx, Y, Cd, prm, X_init=x_init)  # no theta requested
                    outs.append((host(x), host(th), host(x2)))
                tag = f"T={T} init={x_init is not None} graph={graph}"
                np.testing.assert_array_equal(outs[0][0], outs[1][0], err_msg="x " + tag)
                np.testing.assert_array_equal(outs[0][1], outs[1][1], err_msg="theta " + tag)
                np.testing.assert_array_equal(outs[0][2], outs[0][0], err_msg="x without theta " + tag)
    e = rel_l2(outs[0][0], orc.gap_tv(host(Y), C, f32(0.1), 6, 7, tv=tv, x_init=host(x0))[0])
    say(f"GAP-{tv} B={B} {nx}x{ny} {masks}: row and tiled shapes bit-equal; rel-L2 vs oracle {e:.2e}")
    assert e <= REL_TOL
