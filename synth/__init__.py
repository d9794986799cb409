"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module holds no arithmetic of the transform-coding method itself: it only
draws pixels.  The paper measures on natural 8-bit grayscale images and on
video test sequences, none of which ship with it; the separable first-order
Gauss-Markov (AR(1)) field stands in for them because it is the image model the
paper itself uses to score transforms (Sec. 4.2, inter-pixel correlation
rho = 0.95) and the paper reports an average image correlation near 0.86
(Sec. 6.1.2).

Every generator is a pure function of its seed(s): the oracle and the GPU path
receive identical bytes.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.signal import lfilter

__all__ = [
    "ar1_field",
    "ar1_image",
    "BatchImage",
    "batch_specs",
    "batch_images",
    "VideoSpec",
    "video_spec",
    "video_base_planes",
    "video_frame",
    "patch_specs",
    "filter_params",
]


def _ar1_along(x: np.ndarray, rho: float, axis: int) -> np.ndarray:
    """Unit-variance stationary AR(1) recursion along `axis`:
    y[0] = x[0];  y[n] = rho*y[n-1] + sqrt(1-rho^2)*x[n]."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, -1)
    c = math.sqrt(1.0 - rho * rho)
    y = np.empty_like(x)
    y[..., 0] = x[..., 0]
    if x.shape[-1] > 1:
        zi = (rho * x[..., 0])[..., None]
        y[..., 1:], _ = lfilter([c], [1.0, -rho], x[..., 1:], axis=-1, zi=zi)
    return np.moveaxis(y, -1, axis)


def ar1_field(h: int, w: int, rho: float, seed: int) -> np.ndarray:
    """Separable unit-variance AR(1) field: covariance rho^(|di|+|dj|).

    w ~ N(0,1) from numpy's PCG64(seed); the recursion runs along rows first,
    then down the columns of that result."""
    rng = np.random.Generator(np.random.PCG64(seed))
    white = rng.standard_normal((h, w))
    return _ar1_along(_ar1_along(white, rho, axis=1), rho, axis=0)


def ar1_image(h: int, w: int, rho: float = 0.95, seed: int = 0,
              mean: float = 128.0, std: float = 40.0) -> np.ndarray:
    """8-bit grayscale image: clip(rint(mean + std*field), 0, 255) as uint8."""
    f = ar1_field(h, w, rho, seed)
    return np.clip(np.rint(mean + std * f), 0, 255).astype(np.uint8)


# --------------------------------------------------------------------------
# Batched evaluation workload: 45 images of uneven sizes.
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class BatchImage:
    index: int
    h: int
    w: int
    rho: float
    seed: int


def batch_specs(n: int = 45, seed: int = 0) -> list[BatchImage]:
    """n images: W in {256..2048 step 64}, H in {256..1536 step 64},
    rho ~ U[0.85, 0.98]; sizes and rho drawn from PCG64(seed); image i's
    field uses seed i (1-based)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(1, n + 1):
        w = int(rng.integers(256 // 64, 2048 // 64 + 1)) * 64
        h = int(rng.integers(256 // 64, 1536 // 64 + 1)) * 64
        rho = float(rng.uniform(0.85, 0.98))
        out.append(BatchImage(i - 1, h, w, rho, i))
    return out


def batch_images(specs: list[BatchImage]) -> list[np.ndarray]:
    return [ar1_image(s.h, s.w, s.rho, s.seed) for s in specs]


# --------------------------------------------------------------------------
# Video-like stream: YUV 4:2:0 frames, textures translated frame to frame.
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class VideoSpec:
    n_frames: int
    width: int          # luma width
    height: int         # luma height
    rho: float
    seed: int
    margin: int = 4     # luma translation range 0..margin

    @property
    def plane_shapes(self) -> list[tuple[int, int]]:
        """(H, W) of the Y, U, V planes."""
        return [(self.height, self.width),
                (self.height // 2, self.width // 2),
                (self.height // 2, self.width // 2)]

    @property
    def frame_bytes(self) -> int:
        return sum(h * w for h, w in self.plane_shapes)

    @property
    def plane_offsets(self) -> list[int]:
        offs, acc = [], 0
        for h, w in self.plane_shapes:
            offs.append(acc)
            acc += h * w
        return offs

    def offsets(self) -> np.ndarray:
        """Per-frame luma translation (dy, dx), i.i.d. in {0..margin}^2."""
        rng = np.random.Generator(np.random.PCG64(self.seed + 1_000_003))
        return rng.integers(0, self.margin + 1, size=(self.n_frames, 2))


def video_spec(n_frames: int = 300, width: int = 3840, height: int = 2160,
               rho: float = 0.95, seed: int = 7) -> VideoSpec:
    return VideoSpec(n_frames, width, height, rho, seed)


def video_base_planes(spec: VideoSpec) -> list[np.ndarray]:
    """Per-plane base textures, each `margin` pixels larger than the plane,
    with distinct seeds (mean 128, std 40)."""
    m = spec.margin
    return [ar1_image(h + m, w + m, spec.rho, spec.seed * 16 + p)
            for p, (h, w) in enumerate(spec.plane_shapes)]


def video_frame(spec: VideoSpec, bases: list[np.ndarray], f: int) -> np.ndarray:
    """Frame f as one contiguous uint8 buffer: Y, then U, then V (planar).
    Chroma planes move by half the luma translation (floor)."""
    dy, dx = (int(v) for v in spec.offsets()[f])
    parts = []
    for p, (h, w) in enumerate(spec.plane_shapes):
        oy, ox = (dy, dx) if p == 0 else (dy // 2, dx // 2)
        parts.append(np.ascontiguousarray(bases[p][oy:oy + h, ox:ox + w]).ravel())
    return np.concatenate(parts)


# --------------------------------------------------------------------------
# Post-filter training patches.
# --------------------------------------------------------------------------

def patch_specs(n: int, seed: int = 11, size: int = 64,
                field: int = 512, retain=(6, 10, 16)):
    """Patch recipe for the learned post-filter: patch k is cut from AR(1)
    image (k // per_image) on the 8x8 grid; rho ~ U[0.85, 0.98] per image;
    the retention level r is drawn uniformly from `retain`.

    Returns (images, table) where table rows are (image, y0, x0, r)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    per_image = (field // size) ** 2
    n_img = (n + per_image - 1) // per_image
    rhos = rng.uniform(0.85, 0.98, size=n_img)
    images = [ar1_image(field, field, float(rhos[i]), seed * 100_000 + i)
              for i in range(n_img)]
    table = np.empty((n, 4), dtype=np.int64)
    g = field // size
    for k in range(n):
        i, j = divmod(k % per_image, g)
        table[k] = (k // per_image, i * size, j * size,
                    retain[int(rng.integers(0, len(retain)))])
    return images, table


def filter_params(seed: int = 0, last_scale: float = 0.1, bias_scale: float = 0.0) -> np.ndarray:
    """Seeded starting weights for the post-filter, flat float32 in the order
    W1 (32,1,3,3), b1 (32), W2 (32,32,3,3), b2 (32), W3 (1,32,3,3), b3 (1).

    Weights are uniform in +-sqrt(6 / fan_in) (fan_in = 9 input taps times
    input channels), the last layer's scaled by `last_scale` so a fresh filter
    starts close to the identity; biases uniform in +-bias_scale."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for shape, fan_in, scale in (((32, 1, 3, 3), 9, 1.0), ((32,), 0, 0.0),
                                 ((32, 32, 3, 3), 288, 1.0), ((32,), 0, 0.0),
                                 ((1, 32, 3, 3), 288, last_scale), ((1,), 0, 0.0)):
        n = int(np.prod(shape))
        if fan_in:
            lim = math.sqrt(6.0 / fan_in) * scale
        else:
            lim = bias_scale
        parts.append(rng.uniform(-lim, lim, size=n) if lim > 0 else np.zeros(n))
    return np.concatenate(parts).astype(np.float32)
