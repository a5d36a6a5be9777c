"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the oracle tests, the GPU parity tests and the
benchmark.  It holds no arithmetic of the filtering method itself: it only
draws images.  Every generator uses ``numpy.random.default_rng(seed)`` and
draws its random numbers in the order written in its docstring, so a recipe
is reproducible from its description alone.

Layout: planar ``(C, H, W)`` float32, C-contiguous, values in [0, 1].

The paper filters natural color images (Kodak, Barbara, Lena, HD photos),
33/200-band hyperspectral images and noisy color images for nonlocal means
(Sec. III).  None of them is available here; these generators stand in for
them with the same channel counts, value range and piecewise-smooth
structure.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "voronoi_rgb",
    "hyperspectral",
    "batch_sizes",
    "WORKLOADS",
    "workload_input",
]


def _nearest_seed(H: int, W: int, sy: np.ndarray, sx: np.ndarray) -> np.ndarray:
    """Index of the nearest seed for every pixel centre (y+1/2, x+1/2).

    Ties go to the lowest seed index (``argmin`` returns the first minimum).
    """
    lab = np.empty((H, W), dtype=np.int32)
    xs = np.arange(W, dtype=np.float64) + 0.5
    rows = max(1, (1 << 22) // max(1, W * len(sy)))
    for y0 in range(0, H, rows):
        y1 = min(H, y0 + rows)
        ys = np.arange(y0, y1, dtype=np.float64) + 0.5
        dy = ys[:, None, None] - sy[None, None, :]
        dx = xs[None, :, None] - sx[None, None, :]
        lab[y0:y1] = np.argmin(dy * dy + dx * dx, axis=2)
    return lab


def voronoi_rgb(H: int, W: int, seeds: int, noise: float, seed: int,
                return_clean: bool = False):
    """Piecewise-constant random Voronoi color image plus Gaussian noise.

    Draw order from ``default_rng(seed)``:
      1. seed positions, ``uniform(0,1,(seeds,2))`` scaled to [0,H) x [0,W)
         (column 0 is y, column 1 is x);
      2. seed colors, ``uniform(0,1,(seeds,3))``;
      3. noise, ``normal(0, noise, (3,H,W))``.
    Each pixel centre takes the color of its nearest seed (ties: lowest
    index); noise is added, the result clipped to [0,1] and cast to float32.
    """
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 1.0, size=(seeds, 2))
    sy = pos[:, 0] * H
    sx = pos[:, 1] * W
    cols = rng.uniform(0.0, 1.0, size=(seeds, 3))
    lab = _nearest_seed(H, W, sy, sx)
    clean = np.ascontiguousarray(np.transpose(cols[lab], (2, 0, 1)))
    noisy = clean + rng.normal(0.0, noise, size=(3, H, W))
    img = np.clip(noisy, 0.0, 1.0).astype(np.float32)
    if return_clean:
        return img, clean.astype(np.float32)
    return img


def hyperspectral(H: int, W: int, bands: int, endmembers: int, alpha: float,
                  noise: float, seed: int) -> np.ndarray:
    """Linear-mixture hyperspectral cube.

    Bands sit at lambda_t = t/(bands-1).  Endmember m is
    e_m(lambda) = 1/2 + sum_{q=1..4} (a_mq/q) cos(pi q lambda + phi_mq),
    min-max rescaled to [0.1, 0.9].  Each pixel is a Dirichlet(alpha)
    convex mix of the endmembers plus N(0, noise^2), clipped to [0,1].

    Draw order from ``default_rng(seed)``: a ~ U(-1/4,1/4) (endmembers x 4),
    phi ~ U(0, 2 pi) (endmembers x 4), abundances Dirichlet (H*W x
    endmembers, row-major pixels), noise ``normal(0, noise, (bands,H,W))``.
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(-0.25, 0.25, size=(endmembers, 4))
    ph = rng.uniform(0.0, 2.0 * np.pi, size=(endmembers, 4))
    lam = np.arange(bands, dtype=np.float64) / (bands - 1)
    q = np.arange(1, 5, dtype=np.float64)
    e = 0.5 + np.sum((a[:, :, None] / q[None, :, None])
                     * np.cos(np.pi * q[None, :, None] * lam[None, None, :]
                              + ph[:, :, None]), axis=1)
    lo = e.min(axis=1, keepdims=True)
    hi = e.max(axis=1, keepdims=True)
    e = 0.1 + 0.8 * (e - lo) / (hi - lo)
    ab = rng.dirichlet(np.full(endmembers, alpha), size=H * W)
    cube = (ab @ e).T.reshape(bands, H, W)
    cube = cube + rng.normal(0.0, noise, size=(bands, H, W))
    return np.clip(cube, 0.0, 1.0).astype(np.float32)


def lowlight_ir(H: int, W: int, seeds: int, gain: float, noise: float, ir_noise: float,
                seed: int):
    """A dim noisy color image and an infrared channel of the same scene.

    Draw order from ``default_rng(seed)``: the clean scene as in
    :func:`voronoi_rgb` (seed positions, seed colors; no noise draw), then
    ``normal(0, noise, (3,H,W))`` for the color image and
    ``normal(0, ir_noise, (H,W))`` for the infrared one.  The color image is
    gain * clean + noise; the infrared image is the scene's mean over the
    three colors plus its noise (it shares the scene's edges).  Both clipped
    to [0,1], float32; returns (color (3,H,W), infrared (1,H,W)).
    """
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 1.0, size=(seeds, 2))
    cols = rng.uniform(0.0, 1.0, size=(seeds, 3))
    lab = _nearest_seed(H, W, pos[:, 0] * H, pos[:, 1] * W)
    clean = np.transpose(cols[lab], (2, 0, 1))
    low = gain * clean + rng.normal(0.0, noise, size=(3, H, W))
    ir = clean.mean(axis=0) + rng.normal(0.0, ir_noise, size=(H, W))
    return (np.clip(low, 0.0, 1.0).astype(np.float32),
            np.clip(ir, 0.0, 1.0).astype(np.float32)[None])


def voronoi_volume(D: int, H: int, W: int, seeds: int, noise: float, seed: int) -> np.ndarray:
    """Piecewise-constant random 3-D Voronoi vector field (three components)
    plus Gaussian noise: a stand-in for a flow field on a volume.

    Draw order from ``default_rng(seed)``: seed positions
    ``uniform(0,1,(seeds,3))`` scaled to [0,D) x [0,H) x [0,W) (columns z, y,
    x), seed vectors ``uniform(0,1,(seeds,3))``, then noise
    ``normal(0, noise, (3,D,H,W))``.  Each voxel centre takes the vector of its
    nearest seed (ties: lowest index); clipped to [0,1], float32.
    """
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 1.0, size=(seeds, 3)) * np.array([D, H, W], dtype=np.float64)
    vec = rng.uniform(0.0, 1.0, size=(seeds, 3))
    lab = np.empty((D, H, W), dtype=np.int64)
    ys = np.arange(H, dtype=np.float64) + 0.5
    xs = np.arange(W, dtype=np.float64) + 0.5
    for z in range(D):
        dz = (z + 0.5 - pos[:, 0]) ** 2
        for y0 in range(0, H, 64):
            y1 = min(H, y0 + 64)
            d = (dz[None, None, :] + (ys[y0:y1, None, None] - pos[None, None, :, 1]) ** 2
                 + (xs[None, :, None] - pos[None, None, :, 2]) ** 2)
            lab[z, y0:y1] = np.argmin(d, axis=2)
    vol = np.transpose(vec[lab], (3, 0, 1, 2)) + rng.normal(0.0, noise, size=(3, D, H, W))
    return np.clip(vol, 0.0, 1.0).astype(np.float32)


def batch_sizes(count: int = 16, seed: int = 1004):
    """Image sizes of the ragged batch.

    Image 0 is 384x384 and image count-1 is 768x1024; images 1..count-2
    draw H from {384, 416, ..., 768} and then W from {384, 416, ..., 1024}
    with ``default_rng(seed).integers`` (H first, then W, per image).
    """
    rng = np.random.default_rng(seed)
    hs = np.arange(384, 768 + 1, 32)
    ws = np.arange(384, 1024 + 1, 32)
    sizes = [(384, 384)]
    for _ in range(count - 2):
        h = int(hs[rng.integers(0, len(hs))])
        w = int(ws[rng.integers(0, len(ws))])
        sizes.append((h, w))
    sizes.append((768, 1024))
    return sizes


# The five workloads, by name.  sigma_s/S for the Gaussian follows
# S = ceil(3 sigma_s); the box kernel of the nonlocal-means workload is 21x21,
# i.e. S = 10.  ``seed`` seeds the workload's generator.
WORKLOADS = {
    "bf_rgb_256": dict(H=256, W=256, n=3, K=16, sigma_s=3.0, S=9, sigma_r=0.1,
                       spatial="gaussian", seeds=32, noise=0.05, seed=1000),
    "bf_rgb_2048": dict(H=2048, W=2048, n=3, K=32, sigma_s=5.0, S=15, sigma_r=0.12,
                        spatial="gaussian", seeds=256, noise=0.05, seed=1001),
    "bf_hyper_512x32": dict(H=512, W=512, n=32, K=64, sigma_s=4.0, S=12, sigma_r=0.2,
                            spatial="gaussian", seed=1002),
    "nlm_rgb_1024": dict(H=1024, W=1024, n=3, K=32, sigma_s=None, S=10,
                         sigma_r=0.1 * np.sqrt(75.0), spatial="box", seeds=64,
                         noise=0.1, patch=5, dims=16, seed=1003),
    "bf_rgb_batch16": dict(n=3, K=32, sigma_s=3.0, S=9, sigma_r=0.1,
                           spatial="gaussian", seeds=32, noise=0.05, seed=1004),
}


def workload_input(name: str, H: int | None = None, W: int | None = None):
    """The input image of workload ``name`` (its ``seed``).

    ``H``/``W`` override the size (same recipe, same seed) for reduced
    parity cases.  The batch returns a list of images (seeds 1400+b); the
    nonlocal-means workload returns ``(noisy, clean)``.
    """
    cfg = WORKLOADS[name]
    if name == "bf_hyper_512x32":
        return hyperspectral(H or cfg["H"], W or cfg["W"], 32, 5, 0.5, 0.02, cfg["seed"])
    if name == "bf_rgb_batch16":
        return [voronoi_rgb(h, w, cfg["seeds"], cfg["noise"], 1400 + b)
                for b, (h, w) in enumerate(batch_sizes())]
    if name == "nlm_rgb_1024":
        return voronoi_rgb(H or cfg["H"], W or cfg["W"], cfg["seeds"], cfg["noise"], cfg["seed"],
                           return_clean=True)
    return voronoi_rgb(H or cfg["H"], W or cfg["W"], cfg["seeds"], cfg["noise"], cfg["seed"])
