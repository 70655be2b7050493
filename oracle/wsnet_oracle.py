"""FP64 reference of the warm-start network (TEST INFRASTRUCTURE ONLY).

Plain numpy, float64, written from the definitions: a "same" 3x3x3
cross-correlation over (frame, row, column) as 27 shifted slices, ReLU, mean
squared error or the theta-space loss mean((D^T r)^2), and the analytic
backward pass (the transposed convolution is the convolution with the
tap-mirrored kernel and the channel roles swapped).
With ``rounding=True`` the values the GPU stores in bf16 (input, weights,
hidden activations, loss gradient, hidden gradients) are rounded to bf16
(round to nearest even) at the same points, so the GPU can be compared
element by element; with ``rounding=False`` everything stays float64 (used
for the finite-difference pin).

Parameter layout (shared with the library's C ABI): per layer l = 0..3 a
[28][16][16] float32 block, slots 0..26 = taps t = 9(dk+1) + 3(di+1) + (dj+1),
entry [t][out][in]; slot 27, column 0 = bias.

Input channels: c_in = 1 takes the video x alone; c_in = 3 takes x and a base
dual (p_h, p_v), and the prediction is base + network output (the loss and
the projection see the sum).
"""
from __future__ import annotations

import numpy as np

LAYERS = 4
HIDDEN = 16
SLOTS = 28 * 16 * 16


def bf16(a):
    """Round float32 values to bf16 (nearest even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def channels(l, c_out=2, c_in=1):
    cin = c_in if l == 0 else HIDDEN
    cout = c_out if l == LAYERS - 1 else HIDDEN
    return cin, cout


def unpack(params, c_out=2, c_in=1):
    """Padded layout -> list of (W [cout][cin][3][3][3], bias [cout]) in float64."""
    P = np.asarray(params, dtype=np.float32).reshape(LAYERS, 28, 16, 16).astype(np.float64)
    out = []
    for l in range(LAYERS):
        cin, cout = channels(l, c_out, c_in)
        W = np.transpose(P[l, :27, :cout, :cin], (1, 2, 0)).reshape(cout, cin, 3, 3, 3)
        out.append((W.copy(), P[l, 27, :cout, 0].copy()))
    return out


def pack(layers, c_out=2, c_in=1):
    P = np.zeros((LAYERS, 28, 16, 16), dtype=np.float32)
    for l, (W, b) in enumerate(layers):
        cin, cout = channels(l, c_out, c_in)
        P[l, :27, :cout, :cin] = np.transpose(W.reshape(cout, cin, 27), (2, 0, 1))
        P[l, 27, :cout, 0] = b
    return P.ravel()


def conv3d_same(x, W, b=None):
    """y[o] = b[o] + sum_c sum_{dk,di,dj} W[o,c,dk,di,dj] x[c, k+dk-1, i+di-1, j+dj-1] (zero outside)."""
    cin, B, nx, ny = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1)))
    y = np.zeros((W.shape[0], B, nx, ny))
    for dk in range(3):
        for di in range(3):
            for dj in range(3):
                y += np.einsum("oc,cbij->obij", W[:, :, dk, di, dj], xp[:, dk:dk + B, di:di + nx, dj:dj + ny])
    if b is not None:
        y += b[:, None, None, None]
    return y


def conv3d_transposed(dy, W):
    """dx[c] = sum_o sum_t W[o, c, t] dy[o, v - offset(t)]."""
    return conv3d_same(dy, np.transpose(W[:, :, ::-1, ::-1, ::-1], (1, 0, 2, 3, 4)))


def network_input(x, base=None, c_in=1):
    """[c_in][B][nx][ny]: x, then (c_in = 3) the base dual's two fields (zero if None)."""
    x = np.asarray(x, dtype=np.float64)[None]
    if c_in == 1:
        return x
    b = np.zeros((2,) + x.shape[1:]) if base is None else np.asarray(base, dtype=np.float64)
    return np.concatenate([x, b], axis=0)


def forward(x, params, c_out=2, rounding=True, base=None, c_in=1):
    """x [B][nx][ny]; returns (activations a0..a3 [C][B][nx][ny], raw output [c_out][B][nx][ny])."""
    rd = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    layers = unpack(params, c_out, c_in)
    a = [rd(network_input(x, base, c_in))]
    for l, (W, b) in enumerate(layers):
        y = conv3d_same(a[-1], rd(W), b)
        if l < LAYERS - 1:
            a.append(rd(np.maximum(y, 0.0)))
        else:
            return a, y
    raise AssertionError


def dual_adjoint(r):
    """D^T r for a dual r [2][B][nx][ny] (forward differences, no wrap; the
    entries that carry no difference are ignored): per voxel
    (r_h(j-1) - r_h(j)) + (r_v(i-1) - r_v(i)), missing neighbours 0."""
    h = np.array(r[0], dtype=np.float64)
    v = np.array(r[1], dtype=np.float64)
    h[:, :, -1] = 0.0
    v[:, -1, :] = 0.0
    left = np.zeros_like(h)
    left[:, :, 1:] = h[:, :, :-1]
    up = np.zeros_like(v)
    up[:, 1:, :] = v[:, :-1, :]
    return (left - h) + (up - v)


def difference(g):
    """D g [2][B][nx][ny]: g(j+1) - g(j), g(i+1) - g(i), 0 where the
    difference does not exist."""
    g = np.asarray(g, dtype=np.float64)
    out = np.zeros((2,) + g.shape)
    out[0, :, :, :-1] = g[:, :, 1:] - g[:, :, :-1]
    out[1, :, :-1, :] = g[:, 1:, :] - g[:, :-1, :]
    return out


def loss_and_grads(x, target, params, c_out=2, rounding=True, base=None, c_in=1, loss="dual"):
    """loss="dual": MSE 1/(c_out V) sum ((base +) y - target)^2; loss="theta":
    1/V sum (D^T r)^2 with r = (base +) y - target (c_out = 2). Returns the
    loss and the gradient in the padded layout."""
    rd = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    layers = unpack(params, c_out, c_in)
    a, y = forward(x, params, c_out, rounding, base, c_in)
    t = np.asarray(target, dtype=np.float64)
    diff = y - t
    if c_in == 3 and base is not None:
        diff = diff + np.asarray(base, dtype=np.float64)
    if loss == "theta":
        g = dual_adjoint(diff)
        n = g.size
        value = float((g ** 2).sum() / n)
        grad_r = 2.0 * difference(g) / n  # d/dr of sum (D^T r)^2 / n
    else:
        n = t.size
        value = float((diff ** 2).sum() / n)
        grad_r = 2.0 * diff / n
    dy = rd(grad_r) if not rounding else bf16(grad_r.astype(np.float32))
    grads = []
    for l in range(LAYERS - 1, -1, -1):
        W, _ = layers[l]
        ain = a[l]
        dW = np.zeros_like(W)
        ap = np.pad(ain, ((0, 0), (1, 1), (1, 1), (1, 1)))
        B, nx, ny = ain.shape[1:]
        for dk in range(3):
            for di in range(3):
                for dj in range(3):
                    dW[:, :, dk, di, dj] = np.einsum("obij,cbij->oc", dy, ap[:, dk:dk + B, di:di + nx, dj:dj + ny])
        grads.append((dW, dy.sum(axis=(1, 2, 3))))
        if l > 0:
            dx = conv3d_transposed(dy, rd(W))
            dy = rd(dx) * (ain > 0)
    grads.reverse()
    return value, pack(grads, c_out, c_in)


def adam_step(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments), all float64."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def project_dual(raw, tv):
    """Network output [2][B][nx][ny] -> dual-ball projection with the entries
    that carry no difference zeroed (same rule as the denoiser)."""
    p = np.array(raw, dtype=np.float64)
    p[0, :, :, -1] = 0.0
    p[1, :, -1, :] = 0.0
    if tv == "atv":
        return np.clip(p, -1, 1)
    if tv == "itv2d":
        n = np.sqrt(p[0] ** 2 + p[1] ** 2)
    else:
        n = np.sqrt((p[0] ** 2 + p[1] ** 2).sum(axis=0, keepdims=True))
    return p / np.maximum(1.0, n)
