"""Seeded synthetic inputs for the FIO apply.

This module is shared by the CPU oracle's tests, the GPU parity tests and the
benchmark.  It holds only random draws and the input convention of the
problem statement (the 1/N-normalised DFT that turns a grid function f into
f-hat, Section 1.2, eq. (dft)); it contains none of the wedge method's
arithmetic.

Layouts (shared with the C ABI):
  * spatial arrays f, u: shape (N, N), index [n1, n2] for x = (n1/N, n2/N);
  * frequency arrays f-hat: shape (N, N), *centred*: index [k1 + N/2, k2 + N/2]
    for xi = (k1, k2), -N/2 <= k1, k2 < N/2.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng_for", "white_noise_real", "complex_gaussian", "gaussian_bumps",
    "fhat_from_f", "sample_points", "uneven_instances", "training_scales",
    "heldout_scales",
]


def rng_for(config: int, instance: int = 0) -> np.random.Generator:
    """Generator seeded with 1000*config + instance (one stream per input)."""
    return np.random.default_rng(1000 * int(config) + int(instance))


def white_noise_real(N: int, rng: np.random.Generator) -> np.ndarray:
    """i.i.d. real N(0,1) samples on the N x N grid (Section 4 white noise)."""
    return rng.standard_normal((N, N))


def complex_gaussian(N: int, rng: np.random.Generator, B: int | None = None) -> np.ndarray:
    """(N(0,1) + i N(0,1))/sqrt(2) on the grid; shape (B, N, N) if B is given."""
    shape = (N, N) if B is None else (B, N, N)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def gaussian_bumps(N: int, rng: np.random.Generator, count: int = 20) -> np.ndarray:
    """Sum of `count` periodic Gaussian bumps with widths in [1/N, 8/N].

    f(x) = sum_k a_k exp(-d(x, c_k)^2 / (2 w_k^2)), d the minimum-image
    distance on the unit torus, c_k ~ U[0,1)^2, w_k ~ U[1/N, 8/N],
    a_k complex Gaussian.
    """
    n = np.arange(N) / N
    x1, x2 = np.meshgrid(n, n, indexing="ij")
    f = np.zeros((N, N), dtype=np.complex128)
    centres = rng.random((count, 2))
    widths = rng.uniform(1.0 / N, 8.0 / N, size=count)
    amps = (rng.standard_normal(count) + 1j * rng.standard_normal(count)) / np.sqrt(2.0)
    for c, w, a in zip(centres, widths, amps):
        d1 = (x1 - c[0] + 0.5) % 1.0 - 0.5
        d2 = (x2 - c[1] + 0.5) % 1.0 - 0.5
        f += a * np.exp(-(d1 * d1 + d2 * d2) / (2.0 * w * w))
    return f


def fhat_from_f(f: np.ndarray) -> np.ndarray:
    """Centred 1/N-normalised DFT: fhat(xi) = (1/N) sum_x exp(-2 pi i x.xi) f(x).

    Accepts (N, N) or (B, N, N); returns complex128 in the centred layout.
    """
    N = f.shape[-1]
    F = np.fft.fft2(f, axes=(-2, -1)) / N
    return np.fft.fftshift(F, axes=(-2, -1))


def sample_points(N: int, s: int, rng: np.random.Generator) -> np.ndarray:
    """s distinct flat grid indices n1*N + n2, drawn without replacement."""
    s = min(int(s), N * N)
    return np.sort(rng.choice(N * N, size=s, replace=False)).astype(np.int64)


def uneven_instances(count: int = 32, seed: int = 3000):
    """The mixed-size batch: per instance N, phase family, scale and input kind.

    N ~ U{128, 256, 512, 1024}; phase is the c1/c2 ellipse family with a
    scale in [0.5, 1.5] or the rho(x)|xi| family (50/50); the input is a
    complex Gaussian field or a sum of 20 Gaussian bumps (50/50).
    Returns a list of dicts with keys N, family ('c1c2' | 'radial'),
    scale, input ('gaussian' | 'bumps'), seed.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        N = int(rng.choice([128, 256, 512, 1024]))
        family = "c1c2" if rng.random() < 0.5 else "radial"
        scale = float(rng.uniform(0.5, 1.5)) if family == "c1c2" else 1.0
        kind = "gaussian" if rng.random() < 0.5 else "bumps"
        out.append(dict(N=N, family=family, scale=scale, input=kind, seed=seed + 1 + i))
    return out


def instance_field(inst: dict) -> np.ndarray:
    """Spatial input f for one entry of `uneven_instances`."""
    rng = np.random.default_rng(inst["seed"])
    if inst["input"] == "gaussian":
        return complex_gaussian(inst["N"], rng)
    return gaussian_bumps(inst["N"], rng)


def training_scales(count: int = 64) -> np.ndarray:
    """Phase scales s_i = 0.5 + i/(count-1), i = 0..count-1 (spans [0.5, 1.5])."""
    return 0.5 + np.arange(count) / (count - 1.0)


def heldout_scales(count: int = 16) -> np.ndarray:
    """Held-out scales 0.5 + (j + 0.5)/count, j = 0..count-1."""
    return 0.5 + (np.arange(count) + 0.5) / count
