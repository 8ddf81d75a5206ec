"""Seeded synthetic images shaped like the paper's test images.

The paper tests on "a random image" and on piecewise-constant geometric shapes
(Sec. 1, Sec. 3.6); neither is published, so images are generated here.
This module holds no part of the transform's arithmetic: it only draws
pixels, and both the HIP path and the CPU oracle receive what it returns.

cartoon(M, N, n_ellipses, n_halfplanes, sigma, seed):
  background 0; half-planes first, each through a point uniform on the grid
  with a normal angle uniform in [0, 2 pi) and a value uniform in (0, 1),
  painted where (x - p) . n > 0; then ellipses in order (later ones overwrite
  earlier ones), each with centre uniform on the grid, semi-axes uniform in
  (0.02, 0.25) * min(M, N), orientation uniform in [0, pi) and a value
  uniform in (0, 1); finally i.i.d. N(0, sigma^2) noise. Pixels are tested at
  integer coordinates (r, c), without anti-aliasing. Returned as float32.
"""

import numpy as np


def cartoon(M, N, n_ellipses=20, n_halfplanes=10, sigma=0.1, seed=0):
    rng = np.random.default_rng(seed)
    rr, cc = np.meshgrid(np.arange(M, dtype=np.float64),
                         np.arange(N, dtype=np.float64), indexing="ij")
    img = np.zeros((M, N), dtype=np.float64)
    for _ in range(n_halfplanes):
        pr, pc = rng.uniform(0, M), rng.uniform(0, N)
        ang = rng.uniform(0, 2 * np.pi)
        val = rng.uniform(0, 1)
        mask = (rr - pr) * np.cos(ang) + (cc - pc) * np.sin(ang) > 0
        img[mask] = val
    side = min(M, N)
    for _ in range(n_ellipses):
        pr, pc = rng.uniform(0, M), rng.uniform(0, N)
        a = rng.uniform(0.02, 0.25) * side
        b = rng.uniform(0.02, 0.25) * side
        th = rng.uniform(0, np.pi)
        val = rng.uniform(0, 1)
        dr, dc = rr - pr, cc - pc
        u = dr * np.cos(th) + dc * np.sin(th)
        w = -dr * np.sin(th) + dc * np.cos(th)
        img[(u / a) ** 2 + (w / b) ** 2 <= 1.0] = val
    if sigma > 0:
        img = img + rng.normal(0.0, sigma, size=(M, N))
    return img.astype(np.float32)


def gaussian(M, N, seed=0):
    """i.i.d. N(0, 1) image, float32."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((M, N)).astype(np.float32)


def cartoon_batch(M, N, seeds, n_ellipses=20, n_halfplanes=10, sigma=0.1):
    """Stack of cartoons, one per seed, float32 (B, M, N)."""
    return np.stack([cartoon(M, N, n_ellipses, n_halfplanes, sigma, s) for s in seeds])


# Workload recipes with their seeds.
def config1_image():
    """64 x 64, 5 ellipses, noise N(0, 0.05^2), seed 101."""
    return cartoon(64, 64, n_ellipses=5, n_halfplanes=0, sigma=0.05, seed=101)


def config2_image(seed=201):
    """512 x 512, 10 half-planes then 20 ellipses, noise N(0, 0.1^2)."""
    return cartoon(512, 512, n_ellipses=20, n_halfplanes=10, sigma=0.1, seed=seed)


def config2_batch(B=16, first_seed=201):
    return np.stack([config2_image(first_seed + b) for b in range(B)])


def config5_image():
    """2048 x 2048, 200 ellipses, noise N(0, 0.1^2), seed 501."""
    return cartoon(2048, 2048, n_ellipses=200, n_halfplanes=0, sigma=0.1, seed=501)


UNEVEN_SIZES = [(256, 256), (384, 512), (512, 512), (768, 1024), (1024, 1024)]


def uneven_sizes(count=64, seed=401):
    """Image sizes of the uneven batch: drawn uniformly from UNEVEN_SIZES with
    numpy.random.default_rng(seed); J = 3 where the larger side is <= 512,
    else 4. Returns (sizes, Js)."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(UNEVEN_SIZES), size=count)
    sizes = [UNEVEN_SIZES[i] for i in idx]
    return sizes, [3 if max(m, n) <= 512 else 4 for m, n in sizes]


def uneven_images(sizes, first_seed=402):
    """One cartoon per size (10 half-planes, 20 ellipses, noise N(0, 0.1^2)),
    seeds first_seed, first_seed + 1, ..."""
    return [cartoon(m, n, 20, 10, 0.1, first_seed + b) for b, (m, n) in enumerate(sizes)]
