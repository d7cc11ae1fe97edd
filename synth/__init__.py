"""Seeded synthetic inputs for guided linear upsampling.

This module is shared by the oracle tests, the GPU parity tests and the
benchmark.  It produces *inputs only*: high-resolution RGB guide images and
the black-box low-resolution operators ``f`` whose output the upsampler
transfers.  It contains none of the upsampling method's arithmetic (no
downsampling, no pair search, no interpolation).

The paper evaluates on natural-image datasets (an alpha-matting benchmark,
a 2K super-resolution validation set and a dehazing benchmark, Sec. 5.1).
None of them is available here, so these seeded images stand in for them.
They carry the structure the method is sensitive to:

* piecewise-smooth regions: Voronoi cells, each with its own linear colour
  gradient, so that ramps between LR samples exercise the two-colour
  interpolation (Sec. 4.2);
* small isolated dots, the thin or tiny structures that regular-grid
  downsampling drops (Sec. 3.3);
* Gaussian pixel noise;
* colours in [0, 1].

Generator recipe (the constants are this project's, not the paper's):

1. ``rng = numpy.random.default_rng(seed)``.
2. ``n_cells`` sites uniform on a canvas of ``(W + canvas_extra) x H``.
3. Per cell a base colour ``U[0.15, 0.85]^3`` and a gradient matrix
   ``G (3 x 2)`` with entries ``U[-0.3, 0.3] / sqrt(canvas_area / n_cells)``.
4. Pixel colour ``clip(base_k + G_k . ((y, x) - site_k), 0, 1)`` with ``k``
   the nearest site.
5. ``n_dots`` squares of side ``U{lo..hi}`` and colour ``U[0, 1]^3``; a
   placement within 32 px (Chebyshev) of an earlier dot is redrawn.
6. Frame ``t`` is the canvas crop starting at column ``3 t`` (the scene
   translates 3 px per frame).
7. Noise ``N(0, sigma^2)`` per pixel and channel from
   ``default_rng([seed, t])``; clip to [0, 1]; cast to the storage dtype.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "VoronoiScene",
    "voronoi",
    "lr_op_f1",
    "lr_op_f2",
    "COLOR_MATRIX",
    "uneven_batch_specs",
    "noisy_crop_torch",
    "lr_op_f1_torch",
    "video_frames_torch",
    "scene_4k",
    "uneven_batch_torch",
    "SCENE_4K",
    "UNEVEN_CANVAS",
]

# Row-stochastic colour matrix shared by both LR operators: rows are
# non-negative and sum to one, so [0,1]^3 maps into [0,1]^3.
COLOR_MATRIX = np.array(
    [[0.80, 0.15, 0.05], [0.10, 0.80, 0.10], [0.05, 0.15, 0.80]], dtype=np.float64
)

_DOT_SPACING = 32  # Chebyshev distance between dot placements, in HR pixels


@dataclass
class VoronoiScene:
    """A seeded canvas from which frames are cropped (steps 1-5)."""

    H: int
    W: int
    canvas: np.ndarray  # (H, W + canvas_extra, 3) float64, noise-free
    seed: int

    def frame(self, t: int = 0, sigma: float = 0.01, dtype=np.float32) -> np.ndarray:
        """Frame ``t``: crop at column 3t, add seeded noise, clip, cast (steps 6-7)."""
        x0 = 3 * t
        if x0 + self.W > self.canvas.shape[1]:
            raise ValueError("frame %d does not fit the canvas" % t)
        img = self.canvas[:, x0 : x0 + self.W, :]
        if sigma > 0:
            nrng = np.random.default_rng([self.seed, t])
            img = img + sigma * nrng.standard_normal(img.shape)
        img = np.clip(img, 0.0, 1.0)
        return np.ascontiguousarray(img.astype(dtype))


def _nearest_site(H: int, Wc: int, sites: np.ndarray) -> np.ndarray:
    from scipy.spatial import cKDTree

    tree = cKDTree(sites)
    yy, xx = np.mgrid[0:H, 0:Wc]
    pts = np.stack([yy.ravel(), xx.ravel()], axis=1).astype(np.float64)
    out = np.empty(pts.shape[0], dtype=np.int64)
    step = 1 << 21
    for s0 in range(0, pts.shape[0], step):
        _, idx = tree.query(pts[s0 : s0 + step], k=1)
        out[s0 : s0 + step] = idx
    return out.reshape(H, Wc)


def make_scene(
    H: int,
    W: int,
    n_cells: int,
    n_dots: int,
    dot_px=(2, 4),
    seed: int = 0,
    canvas_extra: int = 0,
) -> VoronoiScene:
    rng = np.random.default_rng(seed)
    Wc = W + canvas_extra
    n_cells = max(1, int(n_cells))
    sites = np.stack(
        [rng.uniform(0, H, n_cells), rng.uniform(0, Wc, n_cells)], axis=1
    )  # (y, x)
    base = rng.uniform(0.15, 0.85, size=(n_cells, 3))
    scale = 1.0 / math.sqrt(H * Wc / n_cells)
    grad = rng.uniform(-0.3, 0.3, size=(n_cells, 3, 2)) * scale
    lab = _nearest_site(H, Wc, sites)
    yy, xx = np.mgrid[0:H, 0:Wc]
    dy = yy - sites[lab, 0]
    dx = xx - sites[lab, 1]
    canvas = base[lab] + grad[lab, :, 0] * dy[..., None] + grad[lab, :, 1] * dx[..., None]
    canvas = np.clip(canvas, 0.0, 1.0)

    lo, hi = dot_px
    placed: list[tuple[int, int]] = []
    tries = 0
    while len(placed) < n_dots and tries < 200 * max(1, n_dots):
        tries += 1
        d = int(rng.integers(lo, hi + 1))
        y = int(rng.integers(0, max(1, H - d + 1)))
        x = int(rng.integers(0, max(1, Wc - d + 1)))
        col = rng.uniform(0.0, 1.0, size=3)
        if any(max(abs(y - py), abs(x - px)) < _DOT_SPACING for py, px in placed):
            continue
        placed.append((y, x))
        canvas[y : y + d, x : x + d, :] = col
    return VoronoiScene(H=H, W=W, canvas=canvas, seed=seed)


def voronoi(
    H: int,
    W: int,
    n_cells: int = 64,
    n_dots: int = 20,
    dot_px=(2, 4),
    sigma: float = 0.01,
    seed: int = 0,
    canvas_extra: int = 0,
    t: int = 0,
    dtype=np.float32,
) -> np.ndarray:
    """One seeded H x W x 3 image in [0, 1] (steps 1-7)."""
    scene = make_scene(H, W, n_cells, n_dots, dot_px, seed, canvas_extra)
    return scene.frame(t, sigma=sigma, dtype=dtype)


def lr_op_f1(c: np.ndarray) -> np.ndarray:
    """LR operator f1: colour matrix then gamma 0.8, evaluated in float64.

    ``c`` is (..., 3) in [0, 1]; returns float64 (..., 3) in [0, 1].
    """
    c = np.asarray(c, dtype=np.float64)
    m = np.einsum("ij,...j->...i", COLOR_MATRIX, c)
    return np.power(np.clip(m, 0.0, None), 0.8)


def _gauss5(sigma: float = 1.0) -> np.ndarray:
    x = np.arange(-2, 3, dtype=np.float64)
    g = np.exp(-(x * x) / (2 * sigma * sigma))
    k = np.outer(g, g)
    return k / k.sum()


def lr_op_f2(c: np.ndarray) -> np.ndarray:
    """LR operator f2: 5x5 Gaussian blur (sigma 1, edge-replicate) then the colour matrix.

    ``c`` is (h, w, 3); returns float64 (h, w, 3).
    """
    c = np.asarray(c, dtype=np.float64)
    k = _gauss5(1.0)
    pad = np.pad(c, ((2, 2), (2, 2), (0, 0)), mode="edge")
    h, w = c.shape[:2]
    out = np.zeros_like(c)
    for dy in range(5):
        for dx in range(5):
            out += k[dy, dx] * pad[dy : dy + h, dx : dx + w, :]
    return np.einsum("ij,...j->...i", COLOR_MATRIX, out)


def uneven_batch_specs(n: int = 64, seed: int = 4, wmin=720, wmax=6000, hmin=480, hmax=4000):
    """Shapes, factors and windows of an uneven batch of images.

    Width and height are drawn independently and uniformly, the downsampling
    factor from {4, 8, 16} and the window from {3, 5}.  Cell and dot counts
    scale with the image area (1000 cells and 400 dots at 3840 x 2160).
    Returns a list of dicts with keys H, W, s, k, n_cells, n_dots, seed.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        W = int(rng.integers(wmin, wmax + 1))
        H = int(rng.integers(hmin, hmax + 1))
        s = int(rng.choice([4, 8, 16]))
        k = int(rng.choice([3, 5]))
        area = H * W
        out.append(
            dict(
                H=H,
                W=W,
                s=s,
                k=k,
                n_cells=max(64, int(round(1000 * area / 8.2944e6))),
                n_dots=max(4, int(round(400 * area / 8.2944e6))),
                seed=1000 * seed + i,
            )
        )
    return out


# ---------------------------------------------------------------------------
# Device-resident workloads (torch).  The noise is drawn on the device with
# a seeded torch generator, so the benchmark and the tests that check the
# same launches build bit-identical inputs; neither touches the upsampler.
# ---------------------------------------------------------------------------

# The 4K scene (seed 3, 1000 cells, 400 dots of 1-3 px, 177 extra columns);
# frame t of the 4K video is its canvas crop at column 3 t, with device
# noise seeded 7000 + t
SCENE_4K = dict(H=2160, W=3840, n_cells=1000, n_dots=400, dot_px=(1, 3), seed=3, canvas_extra=177,
                step_x=3, noise_seed0=7000)
# uneven batch: crops of one 6000 x 4000 canvas (seed 4, cell and dot
# density of the 4K scene), crop origins from default_rng(44)
UNEVEN_CANVAS = dict(H=4000, W=6000, n_cells=2894, n_dots=1157, dot_px=(1, 3), seed=4, origin_seed=44)


def noisy_crop_torch(canvas, y0, x0, h, w, seed, dtype, sigma=0.01):
    """A crop of a noise-free canvas (a float32 device tensor) plus seeded
    N(0, sigma^2) noise drawn on the canvas's device, clipped to [0, 1] and
    cast to ``dtype``; contiguous."""
    import torch

    g = torch.Generator(device=canvas.device)
    g.manual_seed(seed)
    img = canvas[y0:y0 + h, x0:x0 + w]
    noise = torch.randn(img.shape, generator=g, device=img.device, dtype=torch.float32)
    return torch.clamp(img + sigma * noise, 0.0, 1.0).to(dtype).contiguous()


def lr_op_f1_torch(c):
    """LR operator f1 (colour matrix, then gamma 0.8) in float32 on the
    tensor's device; returns float32 (..., 3)."""
    import torch

    M = torch.tensor(COLOR_MATRIX, dtype=torch.float32, device=c.device)
    return torch.clamp(c.float() @ M.T, min=0.0) ** 0.8


def scene_4k():
    """The SCENE_4K scene (its canvas and frames)."""
    v = SCENE_4K
    return make_scene(v["H"], v["W"], v["n_cells"], v["n_dots"], v["dot_px"], v["seed"], v["canvas_extra"])


def video_frames_torch(canvas, n, dtype):
    """The ``n`` frames of the 4K video workload as device tensors, from the
    float32 device copy of the SCENE_4K scene's canvas."""
    v = SCENE_4K
    return [noisy_crop_torch(canvas, 0, v["step_x"] * t, v["H"], v["W"], v["noise_seed0"] + t, dtype)
            for t in range(n)]


def uneven_batch_torch(canvas, specs, dtype):
    """The uneven batch's images as device tensors: for each spec a crop of
    the UNEVEN_CANVAS scene's canvas (float32 device copy) at an origin
    drawn from default_rng(origin_seed), with device noise seeded by the
    spec.  Returns the images and their (y0, x0) origins."""
    Hc, Wc = canvas.shape[:2]
    rng = np.random.default_rng(UNEVEN_CANVAS["origin_seed"])
    imgs, origins = [], []
    for sp in specs:
        y0 = int(rng.integers(0, Hc - sp["H"] + 1))
        x0 = int(rng.integers(0, Wc - sp["W"] + 1))
        imgs.append(noisy_crop_torch(canvas, y0, x0, sp["H"], sp["W"], sp["seed"], dtype))
        origins.append((y0, x0))
    return imgs, origins
