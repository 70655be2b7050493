"""Seeded synthetic inputs for video snapshot compressive imaging.

This module only draws random numbers: ground-truth videos, coding masks and
sensor noise. It holds none of the reconstruction arithmetic (no forward
operator, no projection, no TV), so both the FP64 oracle and the HIP library
can consume its arrays without sharing code with each other.

Every array is drawn in float64 from ``numpy.random.default_rng(seed)`` and
rounded once to float32; both sides of a parity test read those float32
values. Layouts follow the measurement model of Sec. 1 (Eq. (3)): a video is
``[B][nx][ny]`` (frame k, row i, column j, column fastest), an image is
``[nx][ny]``.

Scene family (stands in for the paper's simulation videos, which are not
available here): a smooth linear-gradient background plus a number of
piecewise-constant discs / axis-aligned rectangles that translate one pixel
per frame, painted in order with hard edges. Masks are i.i.d. Bernoulli
{0, 1} per voxel, or one Bernoulli base mask shifted by k rows for frame k
(the CACTI-style coding of the paper's references).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = [
    "Problem",
    "scene",
    "masks_bernoulli",
    "masks_shifted",
    "noise_image",
    "make_problem",
    "CONFIGS",
]


def _f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64).astype(np.float32)


def scene(rng: np.random.Generator, nx: int, ny: int, B: int, n_shapes: int = 6,
          radius=(10.0, 40.0), texture_sigma: float = 0.0) -> np.ndarray:
    """Moving piecewise-constant shapes on a gradient background, ``[B][nx][ny]`` float32.

    Background G(i, j) = g0 + g1*i/(nx-1) + g2*j/(ny-1), g0 ~ U[0, 0.2],
    g1, g2 ~ U[0, 0.3]. Each shape is a disc or a rectangle (probability 1/2),
    intensity ~ U[0, 1], radius / half-sides ~ U[radius], centre uniform over
    the image, velocity 1 px/frame along one of +-i, +-j. A static per-pixel
    N(0, texture_sigma^2) texture is added to every frame when requested.
    """
    g0 = rng.uniform(0.0, 0.2)
    g1, g2 = rng.uniform(0.0, 0.3, size=2)
    ii = np.arange(nx, dtype=np.float64)[:, None]
    jj = np.arange(ny, dtype=np.float64)[None, :]
    bg = g0 + g1 * ii / max(nx - 1, 1) + g2 * jj / max(ny - 1, 1)
    vid = np.repeat(bg[None, :, :], B, axis=0)
    dirs = np.array([[1, 0], [-1, 0], [0, 1], [0, -1]], dtype=np.float64)
    for _ in range(n_shapes):
        is_disc = rng.uniform() < 0.5
        val = rng.uniform(0.0, 1.0)
        r1, r2 = rng.uniform(radius[0], radius[1], size=2)
        ci = rng.uniform(0.0, nx)
        cj = rng.uniform(0.0, ny)
        d = dirs[rng.integers(0, 4)]
        for k in range(B):
            pi, pj = ci + k * d[0], cj + k * d[1]
            if is_disc:
                inside = (ii - pi) ** 2 + (jj - pj) ** 2 <= r1 * r1
            else:
                inside = (np.abs(ii - pi) <= r1) & (np.abs(jj - pj) <= r2)
            vid[k][inside] = val
    if texture_sigma > 0.0:
        vid = vid + rng.normal(0.0, texture_sigma, size=(nx, ny))[None, :, :]
    return _f32(vid)


def masks_bernoulli(rng: np.random.Generator, nx: int, ny: int, B: int, p: float = 0.5) -> np.ndarray:
    """i.i.d. Bernoulli(p) {0, 1} coding masks, ``[B][nx][ny]`` float32."""
    return _f32(rng.uniform(size=(B, nx, ny)) < p)


def masks_shifted(rng: np.random.Generator, nx: int, ny: int, B: int, p: float = 0.5) -> np.ndarray:
    """One Bernoulli(p) base mask M; frame k uses M circularly shifted down by k rows."""
    base = rng.uniform(size=(nx, ny)) < p
    return _f32(np.stack([np.roll(base, k, axis=0) for k in range(B)]))


def noise_image(rng: np.random.Generator, nx: int, ny: int, sigma: float) -> np.ndarray:
    """Sensor noise G of Eq. (3): i.i.d. N(0, sigma^2), ``[nx][ny]`` float32 (zeros if sigma == 0)."""
    if sigma <= 0.0:
        return np.zeros((nx, ny), dtype=np.float32)
    return _f32(rng.normal(0.0, sigma, size=(nx, ny)))


@dataclasses.dataclass
class Problem:
    """One synthetic measurement: truth video, masks and noise (the measurement
    itself, Y = sum_k C_k * X_k + G, is formed by whichever side consumes it)."""
    truth: np.ndarray  # [B][nx][ny] float32
    masks: np.ndarray  # [B][nx][ny] float32
    noise: np.ndarray  # [nx][ny] float32
    seed: int
    name: str = ""

    @property
    def dims(self):
        B, nx, ny = self.truth.shape
        return nx, ny, B


def make_problem(nx: int, ny: int, B: int, seed: int, *, mask: str = "bernoulli",
                 mask_p: float = 0.5, sigma: float = 0.0, texture_sigma: float = 0.0,
                 n_shapes: int = 6, radius=(10.0, 40.0), name: str = "") -> Problem:
    """Draw scene, then masks, then noise from one generator seeded with ``seed``."""
    rng = np.random.default_rng(seed)
    truth = scene(rng, nx, ny, B, n_shapes=n_shapes, radius=radius, texture_sigma=texture_sigma)
    if mask == "bernoulli":
        masks = masks_bernoulli(rng, nx, ny, B, mask_p)
    elif mask == "shifted":
        masks = masks_shifted(rng, nx, ny, B, mask_p)
    else:
        raise ValueError(f"unknown mask kind {mask!r}")
    noise = noise_image(rng, nx, ny, sigma)
    return Problem(truth, masks, noise, seed, name)


def batched_specs(n: int = 64, seed: int = 4000):
    """Sizes and coding statistics of a batch of independent measurements:
    nx = ny drawn from {256, 512, 1024}, B from {8, 10, 16}, mask density
    p ~ U[0.3, 0.7], noise sigma ~ U[0, 0.02]. Problem i is drawn with seed
    ``seed + i`` (its own generator, so any subset can be regenerated)."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n):
        side = int(rng.choice([256, 512, 1024]))
        B = int(rng.choice([8, 10, 16]))
        p = float(rng.uniform(0.3, 0.7))
        sigma = float(rng.uniform(0.0, 0.02))
        specs.append(dict(nx=side, ny=side, B=B, seed=seed + i, mask="bernoulli", mask_p=p, sigma=sigma))
    return specs


#: The synthetic workloads, by name. ``lam`` is the TV weight, ``T`` outer and
#: ``N`` inner (FGP) iterations, ``rho`` the ADMM penalty.
CONFIGS = {
    # plain GAP with anisotropic TV on a noiseless 256x256x8 measurement
    "gap_atv_256x8": dict(nx=256, ny=256, B=8, seed=1, mask="bernoulli", sigma=0.0,
                          solver="gap", tv="atv", lam=0.1, T=50, N=5),
    # the six GAP/ADMM x ATV/ITV2D/VTV variants on a noisy 256x256x8 measurement
    "six_256x8": dict(nx=256, ny=256, B=8, seed=2, mask="bernoulli", sigma=0.01,
                      lam=0.1, rho=0.01, T=100, N=10),
    # large CACTI-style measurement: shifted masks, textured scene, GAP-ITV2D
    "cacti_1024x24": dict(nx=1024, ny=1024, B=24, seed=3, mask="shifted", sigma=0.0,
                          texture_sigma=0.02, solver="gap", tv="itv2d", lam=0.1, T=200, N=10),
}


def problem_from_config(name: str, *, nx: Optional[int] = None, ny: Optional[int] = None,
                        B: Optional[int] = None) -> Problem:
    """Regenerate a named workload's inputs (optionally at a smaller size, same recipe)."""
    c = CONFIGS[name]
    return make_problem(nx or c["nx"], ny or c["ny"], B or c["B"], c["seed"], mask=c.get("mask", "bernoulli"),
                        sigma=c.get("sigma", 0.0), texture_sigma=c.get("texture_sigma", 0.0), name=name)
