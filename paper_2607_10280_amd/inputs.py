"""Seeded synthetic inputs shared by the device path, its tests and the benchmark.

This module holds no arithmetic of the method itself: it only draws the inputs that the
feature-extraction problem of §II takes (pixels in [0,1], layer angles, the image-local
pair list of §II-C and the readout parameters of Eq. (4)-(6)).  Everything is a plain
numpy array in float64 / int32; callers convert to device tensors.

Workload recipe (stand-in for the 7x7 downsampled Fashion-MNIST inputs of §II-B and §III,
which are not available here): each image is the clipped sum of 1-3 Gaussian blobs with
centres uniform over the p x p grid, widths sigma ~ U[0.8, 2.5] px and amplitudes
~ U[0.5, 1]; this gives a mostly dark background with a few bright smooth objects and
pixel values in [0, 1].
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


def uniform_pixels(batch: int, n: int, seed: int) -> np.ndarray:
    """Pixels x ~ U[0,1], shape [batch][n], float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 1.0, size=(batch, n))


def blob_image(p: int, seed: int) -> np.ndarray:
    """One p x p Gaussian-blob image flattened row-major (site k = r*p + c), float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = int(rng.integers(1, 4))
    rr, cc = np.meshgrid(np.arange(p, dtype=np.float64), np.arange(p, dtype=np.float64),
                         indexing="ij")
    img = np.zeros((p, p))
    for _ in range(k):
        cy, cx = rng.uniform(0.0, p, size=2)
        sig = rng.uniform(0.8, 2.5)
        amp = rng.uniform(0.5, 1.0)
        img += amp * np.exp(-((rr - cy) ** 2 + (cc - cx) ** 2) / (2.0 * sig * sig))
    return np.clip(img, 0.0, 1.0).reshape(-1)


def blob_images(batch: int, p: int, seed: int) -> np.ndarray:
    """[batch][p*p] Gaussian-blob images; image b uses seed + b."""
    return np.stack([blob_image(p, seed + b) for b in range(batch)])


def layer_angles(n_layers: int, n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """theta, phi ~ U[0, 2pi), each [n_layers][n] float64, shared by a whole batch."""
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = rng.uniform(0.0, TWO_PI, size=(n_layers, n))
    phi = rng.uniform(0.0, TWO_PI, size=(n_layers, n))
    return theta, phi


def neighbour_pairs(p: int, diagonal: bool = False) -> np.ndarray:
    """Image-local pairs of a p x p grid (§II-C): horizontal pairs (k, k+1) in row-major
    order of k, then vertical pairs (k, k+p) in row-major order; int32 [2p(p-1)][2].  With
    `diagonal`, also the diagonal neighbours (r,c)-(r+1,c+1) and then the anti-diagonal ones
    (r,c+1)-(r+1,c), each row-major: 2p(p-1) + 2(p-1)^2 pairs (156 at p = 7, the paper's
    count)."""
    h = [(r * p + c, r * p + c + 1) for r in range(p) for c in range(p - 1)]
    v = [(r * p + c, (r + 1) * p + c) for r in range(p - 1) for c in range(p)]
    d = a = []
    if diagonal:
        d = [(r * p + c, (r + 1) * p + c + 1) for r in range(p - 1) for c in range(p - 1)]
        a = [(r * p + c + 1, (r + 1) * p + c) for r in range(p - 1) for c in range(p - 1)]
    return np.asarray(h + v + d + a, dtype=np.int32).reshape(-1, 2)


def readout_params(m: int, out_dim: int, seed: int, w_std: float = 0.02):
    """Observable parameters A, B (real / imaginary off-diagonal parts, [m][6]) and D
    (diagonal, [m][4]) ~ U[-1, 1], readout weights W ~ N(0, w_std^2) [out_dim][m] and a
    zero bias [out_dim] (§II-A, Eq. (6))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(-1.0, 1.0, size=(m, 6))
    b = rng.uniform(-1.0, 1.0, size=(m, 6))
    d = rng.uniform(-1.0, 1.0, size=(m, 4))
    w = rng.normal(0.0, w_std, size=(out_dim, m))
    bias = np.zeros(out_dim)
    return a, b, d, w, bias


def request_mix(count: int, p_choices, layer_choices, chi_choices, seed: int):
    """Seeded request parameters for mixed batches and serving: for each request (p, L, chi)
    drawn uniformly from the given choices, plus the seeds of its blob image and its angles.
    Returns a list of dicts {p, layers, chi, image_seed, angle_seed}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ps = rng.choice(np.asarray(p_choices), size=count)
    ls = rng.choice(np.asarray(layer_choices), size=count)
    cs = rng.choice(np.asarray(chi_choices), size=count)
    base = int(rng.integers(1 << 30))
    return [{"p": int(ps[i]), "layers": int(ls[i]), "chi": int(cs[i]),
             "image_seed": base + 2 * i, "angle_seed": base + 2 * i + 1} for i in range(count)]


def poisson_arrivals(count: int, qps: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of rate qps: cumulative exponential gaps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / qps, size=count))
