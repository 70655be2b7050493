"""Learned warm start of the FGP denoiser: training data and training loop.

Every step runs in libscitv: the denoiser inputs are the x^(t) that GAP
produces (Eq. (21)) on synthetic measurements, the targets are the duals the
library's own FGP reaches at a tight duality gap, and the network is trained
by the library's MFMA forward/backward kernels and Adam. This module only
orchestrates calls and holds the parameter initialisation.

Two network inputs are supported. c_in = 1 maps x^(t) to a dual. c_in = 3
maps (x^(t), p^(t-1)) to a correction of p^(t-1), the dual the previous outer
iteration ended with (the warm-dual start): its last layer starts at zero, so
the untrained network reproduces the warm-dual start exactly.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np
import torch

from . import scitv

LAYERS = 4
HIDDEN = 16


def channels(l: int, c_out: int = 2, c_in: int = 1):
    return (c_in if l == 0 else HIDDEN), (c_out if l == LAYERS - 1 else HIDDEN)


def init_params(seed: int, c_out: int = 2, last_scale: float = 0.1, c_in: int = 1) -> np.ndarray:
    """He-uniform weights (fan-in 27*cin), zero biases, in the library's padded
    layout [layer][28 slots][16 out][16 in]; the last layer is scaled by
    last_scale (small: an untrained network predicts a small dual; 0 for the
    residual network: it predicts its base dual)."""
    rng = np.random.default_rng(seed)
    P = np.zeros((LAYERS, 28, 16, 16), dtype=np.float32)
    for l in range(LAYERS):
        cin, cout = channels(l, c_out, c_in)
        bound = np.sqrt(6.0 / (27 * cin)) * (last_scale if l == LAYERS - 1 else 1.0)
        P[l, :27, :cout, :cin] = rng.uniform(-bound, bound, size=(27, cout, cin))
    return P.ravel()


def gap_denoiser_inputs(h, Y, C, tv: str, lam: float, n_inner: int, outer: List[int]) -> List[torch.Tensor]:
    """The denoiser inputs x^(t) of a GAP run with n_inner FGP iterations, at
    the listed outer iterations t (1-based)."""
    one = scitv.solver_params(outer_iters=1, tv=tv, lam=lam, n_inner=n_inner)
    theta = scitv.sci_adjoint(h, C, Y)
    x = torch.empty_like(theta)
    nxt = torch.empty_like(theta)
    keep = []
    for t in range(1, max(outer) + 1):
        scitv.sci_gap_tv(h, Y, C, one, X_out=x, Theta_out=nxt, X_init=theta)
        theta, nxt = nxt, theta
        if t in outer:
            keep.append(x.clone())
    return keep


def converged_dual(h, x: torch.Tensor, tv: str, lam: float, tol: float = 1e-6, cap: int = 4000) -> torch.Tensor:
    """The dual FGP reaches at relative duality gap <= tol (cold start)."""
    prm = scitv.tv_params(tv=tv, lam=lam, gap_tol=tol, n_inner_max=cap, gap_check_every=20)
    dual = torch.empty((2,) + tuple(x.shape), device=x.device)
    scitv.sci_tv_denoise(h, x, prm, dual_out=dual, want_gap=True)
    return dual


def warm_dual_triples(h, Y, C, tv: str, lam: float, outer: int, tol: float = 1e-4, target_tol: float = 1e-6,
                      every: int = 1, cap: int = 4000) -> List[Tuple[torch.Tensor, torch.Tensor, torch.Tensor]]:
    """Training data for the c_in = 3 network from one measurement: a
    gap-controlled GAP run with warm duals (each denoiser call starts from the
    previous call's final dual and stops at relative gap tol), recording at
    every `every`-th outer iteration (x^(t), p^(t-1), the dual at target_tol
    for x^(t)). p^(0) = 0."""
    proj = scitv.solver_params(outer_iters=1, tv=tv, lam=lam, n_inner=0)
    at_tol = scitv.tv_params(tv=tv, lam=lam, gap_tol=tol, n_inner_max=cap, gap_check_every=1)
    tight = scitv.tv_params(tv=tv, lam=lam, gap_tol=target_tol, n_inner_max=cap, gap_check_every=20)
    theta = scitv.sci_adjoint(h, C, Y)
    x = torch.empty_like(theta)
    scratch = torch.empty_like(theta)
    prev = torch.zeros((2,) + tuple(theta.shape), device=theta.device)
    out = []
    for t in range(1, outer + 1):
        scitv.sci_gap_tv(h, Y, C, proj, X_out=x, Theta_out=scratch, X_init=theta)  # x^(t), Eq. (21)
        dual = torch.empty_like(prev)
        theta = torch.empty_like(x)
        scitv.sci_tv_denoise(h, x, at_tol, Theta_out=theta, dual_init=prev, dual_out=dual)
        if t % every == 0:
            target = torch.empty_like(prev)
            scitv.sci_tv_denoise(h, x, tight, dual_init=dual, dual_out=target)
            out.append((x.clone(), prev, target))
        prev = dual
    return out


class CropSet:
    """Training examples stored as crops of full-frame solves, all frames of a
    crop x crop window: X [n][B][c][c] (denoiser inputs x^(t)), P [n][2][B][c][c]
    (the previous outer iteration's final dual, the base of the correcting
    network) and T [n][2][B][c][c] (the dual FGP reaches at a tight gap).
    Preallocated on the device for `capacity` crops."""

    def __init__(self, capacity: int, B: int, crop: int, device):
        self.X = torch.empty((capacity, B, crop, crop), device=device)
        self.P = torch.empty((capacity, 2, B, crop, crop), device=device)
        self.T = torch.empty((capacity, 2, B, crop, crop), device=device)
        self.n = 0
        self.crop = crop

    def add_frame(self, x: torch.Tensor, base: torch.Tensor, target: torch.Tensor) -> int:
        """Cut one full-frame example into crop x crop windows on a regular grid
        (as many as fit, and as the capacity allows); returns the crops added."""
        c = self.crop
        _, nx, ny = x.shape
        added = 0
        for i0 in range(0, nx - c + 1, c):
            for j0 in range(0, ny - c + 1, c):
                if self.n == self.X.shape[0]:
                    return added
                self.X[self.n].copy_(x[:, i0:i0 + c, j0:j0 + c])
                self.P[self.n].copy_(base[:, :, i0:i0 + c, j0:j0 + c])
                self.T[self.n].copy_(target[:, :, i0:i0 + c, j0:j0 + c])
                self.n += 1
                added += 1
        return added

    def example(self, i: int, with_base: bool):
        return (self.X[i], self.P[i], self.T[i]) if with_base else (self.X[i], self.T[i])


def fill_crop_set(h, cs: CropSet, Y, C, tv: str, lam: float, outer: int, tol: float = 1e-4,
                  target_tol: float = 1e-6, cap: int = 4000, every: int = 5) -> int:
    """Add the crops of one measurement: a gap-controlled GAP run with warm duals
    (each denoiser call starts from the previous call's final dual and stops at
    relative gap tol, checked every `every` iterations); at every outer
    iteration t, x^(t), p^(t-1) and the dual at target_tol for x^(t) (started
    from the tol dual) are cut into crops. p^(0) = 0. Returns the crops added."""
    proj = scitv.solver_params(outer_iters=1, tv=tv, lam=lam, n_inner=0)
    at_tol = scitv.tv_params(tv=tv, lam=lam, gap_tol=tol, n_inner_max=cap, gap_check_every=every)
    tight = scitv.tv_params(tv=tv, lam=lam, gap_tol=target_tol, n_inner_max=cap, gap_check_every=20)
    theta = scitv.sci_adjoint(h, C, Y)
    x = torch.empty_like(theta)
    scratch = torch.empty_like(theta)
    prev = torch.zeros((2,) + tuple(theta.shape), device=theta.device)
    dual = torch.empty_like(prev)
    target = torch.empty_like(prev)
    added = 0
    for _ in range(outer):
        scitv.sci_gap_tv(h, Y, C, proj, X_out=x, Theta_out=scratch, X_init=theta)  # x^(t), Eq. (21)
        scitv.sci_tv_denoise(h, x, at_tol, Theta_out=theta, dual_init=prev, dual_out=dual)
        scitv.sci_tv_denoise(h, x, tight, dual_init=dual, dual_out=target)
        added += cs.add_frame(x, prev, target)
        prev, dual = dual, prev
    return added


def mean_loss(h, net, cs: CropSet, idx, with_base: bool) -> float:
    """Mean loss of the network over the listed examples (no update)."""
    tot = 0.0
    for i in idx:
        ex = cs.example(int(i), with_base)
        x, base, t = ex if with_base else (ex[0], None, ex[1])
        loss, _ = scitv.sci_wsnet_grads(h, net, x, t, base=base)
        tot += loss
    return tot / max(1, len(idx))


def train_epochs(h, net, cs: CropSet, with_base: bool, epochs: int, lr: float, held: CropSet = None,
                 n_held: int = 256, log_every: int = 2000, seed: int = 0, progress=None):
    """Adam over the whole crop set in a fresh random order every epoch.
    Returns [(step, mean training loss over the steps since the last entry,
    mean held-out loss)]; the held-out loss is computed on the first n_held
    examples of `held` (no update)."""
    rng = np.random.default_rng(seed)
    hist = []
    step, acc, cnt = 0, 0.0, 0
    hidx = range(min(n_held, held.n)) if held is not None else []
    if held is not None:
        hist.append((0, None, mean_loss(h, net, held, hidx, with_base)))
    for ep in range(epochs):
        for i in rng.permutation(cs.n):
            ex = cs.example(int(i), with_base)
            x, base, t = ex if with_base else (ex[0], None, ex[1])
            acc += scitv.sci_wsnet_train_step(h, net, x, t, lr, base=base, want_loss=True)
            cnt += 1
            step += 1
            if step % log_every == 0 or step == epochs * cs.n:
                ho = mean_loss(h, net, held, hidx, with_base) if held is not None else None
                hist.append((step, acc / cnt, ho))
                if progress:
                    progress(f"step {step}: train loss {acc / cnt:.5f}" + (f", held-out {ho:.5f}" if ho is not None
                                                                           else ""))
                acc, cnt = 0.0, 0
    return hist


def crops(x: torch.Tensor, size: int, n: int, rng: np.random.Generator) -> List[Tuple[int, int]]:
    _, nx, ny = x.shape
    return [(int(rng.integers(0, nx - size + 1)), int(rng.integers(0, ny - size + 1))) for _ in range(n)]


def train(h, net, pairs, steps: int, lr: float = 2e-3, seed: int = 0, log_every: int = 0):
    """Adam on randomly drawn (input, target) or (input, base dual, target)
    examples; returns the loss history."""
    rng = np.random.default_rng(seed)
    hist = []
    for s in range(steps):
        ex = pairs[int(rng.integers(0, len(pairs)))]
        x, base, t = ex if len(ex) == 3 else (ex[0], None, ex[1])
        want = log_every > 0 and (s % log_every == 0 or s == steps - 1)
        loss = scitv.sci_wsnet_train_step(h, net, x, t, lr, base=base, want_loss=want)
        if want:
            hist.append((s, loss))
    return hist
