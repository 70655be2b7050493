"""Pins for the FP64 network oracle: the convolution against scipy's
cross-correlation, the analytic backward pass against central finite
differences, the parameter layout, the Adam update and the dual projection."""
import numpy as np
import pytest
import scipy.signal

from oracle import wsnet_oracle as wo


def rand_params(seed, scale=0.3, c_out=2, c_in=1):
    r = np.random.default_rng(seed)
    layers = []
    for l in range(wo.LAYERS):
        cin, cout = wo.channels(l, c_out, c_in)
        layers.append((r.normal(scale=scale / np.sqrt(27 * cin), size=(cout, cin, 3, 3, 3)),
                       r.normal(scale=0.05, size=cout)))
    return wo.pack(layers, c_out, c_in), layers


def test_conv_matches_scipy_correlate():
    r = np.random.default_rng(0)
    x = r.normal(size=(3, 4, 7, 9))
    W = r.normal(size=(2, 3, 3, 3, 3))
    b = r.normal(size=2)
    y = wo.conv3d_same(x, W, b)
    for o in range(2):
        ref = sum(scipy.signal.correlate(x[c], W[o, c], mode="same", method="direct") for c in range(3)) + b[o]
        np.testing.assert_allclose(y[o], ref, rtol=1e-12, atol=1e-12)


def test_transposed_conv_is_adjoint():
    r = np.random.default_rng(1)
    x = r.normal(size=(3, 4, 6, 5))
    dy = r.normal(size=(2, 4, 6, 5))
    W = r.normal(size=(2, 3, 3, 3, 3))
    lhs = (wo.conv3d_same(x, W) * dy).sum()
    rhs = (x * wo.conv3d_transposed(dy, W)).sum()
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_pack_unpack_round_trip():
    P, layers = rand_params(2)
    back = wo.unpack(P)
    for (W, b), (W2, b2) in zip(layers, back):
        np.testing.assert_allclose(W2, W.astype(np.float32), rtol=0, atol=0)
        np.testing.assert_allclose(b2, b.astype(np.float32), rtol=0, atol=0)


def test_zero_net_gives_zero_dual():
    x = np.random.default_rng(3).uniform(size=(2, 5, 6))
    _, y = wo.forward(x, np.zeros(4 * wo.SLOTS, np.float32))
    assert np.all(y == 0.0)


@pytest.mark.parametrize("c_in", [1, 3])
def test_backward_matches_finite_differences(c_in):
    r = np.random.default_rng(4)
    P, _ = rand_params(5, scale=1.0, c_in=c_in)
    x = r.uniform(size=(2, 5, 6))
    t = r.normal(scale=0.3, size=(2, 2, 5, 6))
    base = r.normal(scale=0.5, size=(2, 2, 5, 6)) if c_in == 3 else None
    loss, g = wo.loss_and_grads(x, t, P, rounding=False, base=base, c_in=c_in)
    assert abs(loss - _loss64(x, t, P.astype(np.float64), base, c_in)) <= 1e-12 * loss
    P64 = P.astype(np.float64)
    live = np.flatnonzero(wo.pack(wo.unpack(np.ones_like(P), c_in=c_in), c_in=c_in) != 0)
    for idx in r.choice(live, size=25, replace=False):
        h = 1e-4 * max(1.0, abs(P64[idx]))

        def f(delta):
            Q = P64.copy()
            Q[idx] += delta
            # evaluate in float64: go through unpack without the float32 cast
            return _loss64(x, t, Q, base, c_in)
        fd = (f(h) - f(-h)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-5 * max(1e-3, abs(fd)), (idx, fd, g[idx])


def _loss64(x, t, Q, base=None, c_in=1):
    """The loss written out independently: the input channels stacked by hand,
    the prediction = base + output for c_in = 3."""
    layers = []
    P = Q.reshape(wo.LAYERS, 28, 16, 16)
    for l in range(wo.LAYERS):
        cin, cout = wo.channels(l, 2, c_in)
        W = np.transpose(P[l, :27, :cout, :cin], (1, 2, 0)).reshape(cout, cin, 3, 3, 3)
        layers.append((W, P[l, 27, :cout, 0]))
    a = np.stack([np.asarray(x, dtype=np.float64)] + ([base[0], base[1]] if c_in == 3 else []))
    for l, (W, b) in enumerate(layers):
        y = wo.conv3d_same(a, W, b)
        a = np.maximum(y, 0.0) if l < wo.LAYERS - 1 else y
    if c_in == 3:
        a = a + base
    return float(((a - t) ** 2).sum() / t.size)


def test_zero_last_layer_predicts_the_base():
    """With c_in = 3 and a zero last layer the prediction is the base dual, so
    the loss is the base's squared distance to the target."""
    r = np.random.default_rng(8)
    P, _ = rand_params(9, c_in=3)
    Q = P.reshape(wo.LAYERS, 28, 16, 16).copy()
    Q[-1] = 0.0
    x = r.uniform(size=(2, 4, 5))
    base = r.normal(size=(2, 2, 4, 5))
    t = r.normal(size=(2, 2, 4, 5))
    _, y = wo.forward(x, Q.ravel(), base=base, c_in=3, rounding=False)
    assert np.all(y == 0.0)
    loss, g = wo.loss_and_grads(x, t, Q.ravel(), rounding=False, base=base, c_in=3)
    assert abs(loss - ((base - t) ** 2).mean()) <= 1e-14
    # only the last layer moves first: the hidden layers see a zero back-propagated gradient
    G = g.reshape(wo.LAYERS, 28, 16, 16)
    assert np.all(G[:-1] == 0.0) and np.any(G[-1] != 0.0)


def test_adam_first_step_is_signed_lr():
    w = np.array([0.5, -0.2, 1.0])
    g = np.array([3.0, -1e-3, 0.0])
    w1, m, v = wo.adam_step(w, g, np.zeros(3), np.zeros(3), 1, 0.01)
    np.testing.assert_allclose(w1[:2], w[:2] - 0.01 * np.sign(g[:2]), rtol=0, atol=1e-7)
    assert w1[2] == w[2]


@pytest.mark.parametrize("tv", ["atv", "itv2d", "vtv"])
def test_project_dual_feasible(tv):
    raw = np.random.default_rng(6).normal(scale=3, size=(2, 3, 4, 5))
    p = wo.project_dual(raw, tv)
    assert np.all(p[0, :, :, -1] == 0) and np.all(p[1, :, -1, :] == 0)
    if tv == "atv":
        assert np.abs(p).max() <= 1
    elif tv == "itv2d":
        assert np.sqrt(p[0] ** 2 + p[1] ** 2).max() <= 1 + 1e-12
    else:
        assert np.sqrt((p ** 2).sum(axis=(0, 1))).max() <= 1 + 1e-12


def test_bf16_rounding_is_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9, -2.5], np.float32)
    # 1 + 2^-8 is the tie between 1 and 1 + 2^-7 (bf16 spacing at 1): even mantissa wins
    np.testing.assert_array_equal(wo.bf16(vals), [1.0, 1.0, 1.0, 1.0 + 2 ** -7, -2.5])


# ---- theta-space loss -------------------------------------------------------

def _difference_matrix(B, nx, ny):
    """D as an explicit matrix, built entry by entry from the forward
    differences: rows = the dual entries that carry a difference (h at
    j < ny-1, then v at i < nx-1), columns = voxels; also the row index of
    each dual entry [2][B][nx][ny] (or -1)."""
    V = B * nx * ny
    vox = lambda b, i, j: (b * nx + i) * ny + j
    rows, where = [], -np.ones((2, B, nx, ny), dtype=np.int64)
    for b in range(B):
        for i in range(nx):
            for j in range(ny):
                if j < ny - 1:
                    where[0, b, i, j] = len(rows)
                    rows.append((vox(b, i, j + 1), vox(b, i, j)))
    for b in range(B):
        for i in range(nx):
            for j in range(ny):
                if i < nx - 1:
                    where[1, b, i, j] = len(rows)
                    rows.append((vox(b, i + 1, j), vox(b, i, j)))
    D = np.zeros((len(rows), V))
    for k, (plus, minus) in enumerate(rows):
        D[k, plus] += 1.0
        D[k, minus] -= 1.0
    return D, where


def _theta_loss_explicit(r, D, where):
    vec = np.array([r[c][tuple(idx)] for c in range(2) for idx in np.argwhere(where[c] >= 0)])
    order = np.concatenate([where[c][where[c] >= 0] for c in range(2)])
    e = np.zeros(D.shape[0])
    e[order] = vec
    g = D.T @ e
    return float((g ** 2).sum() / D.shape[1])


def test_theta_loss_pins():
    """dual_adjoint is D^T and difference is D (adjoint pair, explicit
    matrix); the loss ignores the null space of D^T and the entries that carry
    no difference; a unit error on one inner h entry costs exactly 2/V."""
    r = np.random.default_rng(21)
    B, nx, ny = 2, 4, 5
    D, where = _difference_matrix(B, nx, ny)
    rr = r.normal(size=(2, B, nx, ny))
    g = r.normal(size=(B, nx, ny))
    # <D^T r, g> = <r, D g> with r restricted to the existing entries
    lhs = float((wo.dual_adjoint(rr) * g).sum())
    rm = rr.copy()
    rm[0, :, :, -1] = 0.0
    rm[1, :, -1, :] = 0.0
    assert abs(lhs - float((rm * wo.difference(g)).sum())) <= 1e-12 * max(1.0, abs(lhs))
    assert abs(float((wo.dual_adjoint(rr) ** 2).sum() / g.size) - _theta_loss_explicit(rr, D, where)) <= 1e-12
    # null space of D^T: a target moved along it leaves the loss unchanged
    import scipy.linalg
    N = scipy.linalg.null_space(D.T)
    assert N.shape[1] > 0
    P, _ = rand_params(3, scale=1.0, c_in=3)
    x = r.uniform(size=(B, nx, ny))
    base = r.normal(scale=0.5, size=(2, B, nx, ny))
    t = r.normal(scale=0.3, size=(2, B, nx, ny))
    move = np.zeros_like(t)
    nvec = N @ r.normal(size=N.shape[1])
    for c in range(2):
        idx = np.argwhere(where[c] >= 0)
        move[c][tuple(idx.T)] = nvec[where[c][where[c] >= 0]]
    move[0, :, :, -1] = 5.0  # entries without a difference do not count either
    l0, _ = wo.loss_and_grads(x, t, P, rounding=False, base=base, c_in=3, loss="theta")
    l1, _ = wo.loss_and_grads(x, t + move, P, rounding=False, base=base, c_in=3, loss="theta")
    assert abs(l0 - l1) <= 1e-12 * l0
    # closed form: one unit error at an inner h entry
    e = np.zeros((2, B, nx, ny))
    e[0, 1, 2, 1] = 1.0
    assert abs(float((wo.dual_adjoint(e) ** 2).sum()) / (B * nx * ny) - 2.0 / (B * nx * ny)) <= 1e-15


@pytest.mark.parametrize("c_in", [1, 3])
def test_theta_loss_gradient_matches_finite_differences(c_in):
    r = np.random.default_rng(8)
    P, _ = rand_params(9, scale=1.0, c_in=c_in)
    B, nx, ny = 2, 5, 6
    x = r.uniform(size=(B, nx, ny))
    t = r.normal(scale=0.3, size=(2, B, nx, ny))
    base = r.normal(scale=0.5, size=(2, B, nx, ny)) if c_in == 3 else None
    D, where = _difference_matrix(B, nx, ny)
    loss, g = wo.loss_and_grads(x, t, P, rounding=False, base=base, c_in=c_in, loss="theta")
    P64 = P.astype(np.float64)

    def explicit(Q):
        layers = []
        W4 = Q.reshape(wo.LAYERS, 28, 16, 16)
        for l in range(wo.LAYERS):
            cin, cout = wo.channels(l, 2, c_in)
            W = np.transpose(W4[l, :27, :cout, :cin], (1, 2, 0)).reshape(cout, cin, 3, 3, 3)
            layers.append((W, W4[l, 27, :cout, 0]))
        a = np.stack([x] + ([base[0], base[1]] if c_in == 3 else []))
        for l, (W, b) in enumerate(layers):
            yy = wo.conv3d_same(a, W, b)
            a = np.maximum(yy, 0.0) if l < wo.LAYERS - 1 else yy
        pred = a + base if c_in == 3 else a
        return _theta_loss_explicit(pred - t, D, where)

    assert abs(loss - explicit(P64)) <= 1e-12 * loss
    live = np.flatnonzero(wo.pack(wo.unpack(np.ones_like(P), c_in=c_in), c_in=c_in) != 0)
    last = live[live >= (wo.LAYERS - 1) * wo.SLOTS]
    # the loss is quadratic in the last layer's parameters: central differences
    # are exact there; in the hidden layers a small step keeps clear of the
    # ReLU kinks
    for idx, h, tol in [(i, 1e-3, 1e-8) for i in r.choice(last, size=10, replace=False)] + \
                       [(i, 1e-6, 2e-3) for i in r.choice(live[live < (wo.LAYERS - 1) * wo.SLOTS], size=10,
                                                           replace=False)]:
        Qp, Qm = P64.copy(), P64.copy()
        Qp[idx] += h
        Qm[idx] -= h
        fd = (explicit(Qp) - explicit(Qm)) / (2 * h)
        assert abs(fd - g[idx]) <= tol * max(1e-3, abs(fd)), (idx, fd, g[idx])
