"""Seeded synthetic scene generators (inputs only).

The paper builds its own 2-D test scenes and publishes none of them (Section 5),
so every workload here is synthetic: per-pixel emission ``eps`` (radiance added
per unit length, the integrand of Eq. 3) and attenuation ``sigma`` (sigma_t of
Eq. 2) on a square grid, each pixel a square of uniform medium (Section 5).

This module is shared by the tests, the benchmark and the oracle's callers.  It
holds no part of the method's arithmetic: it only draws random shapes.

Generation order for every recipe: ``rng = numpy.random.default_rng(seed)``,
then fog, then boxes, then lines (each sets sigma, overriding what was there),
then disks (each sets eps, overriding; sigma unchanged).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "Scene", "value_noise", "add_box", "add_disk", "add_line",
    "config1", "config2", "config3", "config4", "config5", "scene_like_512",
]


@dataclass
class Scene:
    eps: np.ndarray    # [S][S] float32, row-major (row r, column c)
    sigma: np.ndarray  # [S][S] float32
    seed: int
    name: str

    @property
    def size(self) -> int:
        return self.eps.shape[0]


def value_noise(rng: np.random.Generator, S: int, octaves: int = 4) -> np.ndarray:
    """Sum of ``octaves`` value-noise layers in [0, 1].

    Octave o has lattice period S/(8*2^o) pixels (at least 1), uniform lattice
    values in [0,1), smoothstep-weighted bilinear interpolation evaluated at pixel
    centres, and amplitude 2^-o.  The sum is divided by the total amplitude so it
    stays in [0, 1].
    """
    out = np.zeros((S, S), dtype=np.float64)
    total = 0.0
    for o in range(octaves):
        period = max(S / (8.0 * 2 ** o), 1.0)
        cells = int(np.ceil(S / period))
        lat = rng.random((cells + 1, cells + 1))
        t = (np.arange(S) + 0.5) / period
        i0 = np.minimum(np.floor(t).astype(np.int64), cells - 1)
        f = t - i0
        s = f * f * (3.0 - 2.0 * f)
        a = lat[i0][:, i0]
        b = lat[i0][:, i0 + 1]
        c = lat[i0 + 1][:, i0]
        d = lat[i0 + 1][:, i0 + 1]
        sr = s[:, None]
        sc = s[None, :]
        layer = (a * (1 - sc) + b * sc) * (1 - sr) + (c * (1 - sc) + d * sc) * sr
        amp = 2.0 ** (-o)
        out += amp * layer
        total += amp
    return out / total


def add_box(rng: np.random.Generator, field: np.ndarray, side_lo: int, side_hi: int,
            value) -> None:
    """Axis-aligned box with integer corners, sides uniform in {side_lo..side_hi}
    (clipped to the grid side).

    ``value`` is a float, or the string ``"u05"`` for per-pixel U[0,5] values.
    """
    S = field.shape[0]
    h = min(int(rng.integers(side_lo, side_hi + 1)), S)
    w = min(int(rng.integers(side_lo, side_hi + 1)), S)
    r0 = int(rng.integers(0, S - h + 1))
    c0 = int(rng.integers(0, S - w + 1))
    if isinstance(value, str):
        field[r0:r0 + h, c0:c0 + w] = rng.uniform(0.0, 5.0, size=(h, w))
    else:
        field[r0:r0 + h, c0:c0 + w] = value


def add_line(rng: np.random.Generator, field: np.ndarray, horizontal: bool,
             len_lo: int, len_hi: int, value: float) -> None:
    """One-pixel-wide axis-aligned line of the given sigma."""
    S = field.shape[0]
    n = int(rng.integers(len_lo, len_hi + 1))
    a = int(rng.integers(0, S - n + 1))
    b = int(rng.integers(0, S))
    if horizontal:
        field[b, a:a + n] = value
    else:
        field[a:a + n, b] = value


def add_disk(rng: np.random.Generator, field: np.ndarray, r_lo: float, r_hi: float,
             value: float) -> None:
    """Disk of radius rho ~ U[r_lo, r_hi] (at most S/4), centre uniform in [rho, S-rho]^2.

    Pixel (r, c) is covered iff its centre lies within rho of the disk centre.
    """
    S = field.shape[0]
    rho = min(float(rng.uniform(r_lo, r_hi)), S / 4.0)
    cx = float(rng.uniform(rho, S - rho))
    cy = float(rng.uniform(rho, S - rho))
    r = np.arange(S) + 0.5
    mask = (r[None, :] - cx) ** 2 + (r[:, None] - cy) ** 2 <= rho * rho
    field[mask] = value


def _loguniform(rng: np.random.Generator, lo: float, hi: float) -> float:
    return float(np.exp(rng.uniform(np.log(lo), np.log(hi))))


def config1(seed: int = 1) -> Scene:
    """64x64: 3 disks (radius 2-6, eps ~ U[1,10]); 4 boxes (sides 4-16) of
    per-pixel sigma ~ U[0,5]; zero elsewhere."""
    S = 64
    rng = np.random.default_rng(seed)
    eps = np.zeros((S, S))
    sig = np.zeros((S, S))
    for _ in range(4):
        add_box(rng, sig, 4, 16, "u05")
    for _ in range(3):
        add_disk(rng, eps, 2.0, 6.0, float(rng.uniform(1.0, 10.0)))
    return Scene(eps.astype(np.float32), sig.astype(np.float32), seed, "disks3_boxes4_64")


def scene_like_512(S: int, seed: int, n_disks: int, n_boxes: int, n_lines: int = 0,
                   box_sigma=50.0, fog: float = 0.05, name: str = "") -> Scene:
    """Fog of sigma = fog * 4-octave value noise, ``n_boxes`` boxes (sides 4-16)
    of sigma ``box_sigma``, ``n_lines`` one-pixel lines of sigma 100 (half
    horizontal, half vertical, length 64-256 clipped to the grid), and
    ``n_disks`` disks (radius 2-12, eps log-uniform on [0.5, 50])."""
    rng = np.random.default_rng(seed)
    eps = np.zeros((S, S))
    sig = fog * value_noise(rng, S) if fog > 0 else np.zeros((S, S))
    for _ in range(n_boxes):
        add_box(rng, sig, 4, 16, box_sigma)
    for i in range(n_lines):
        add_line(rng, sig, i < n_lines // 2, min(64, S), min(256, S), 100.0)
    for _ in range(n_disks):
        add_disk(rng, eps, 2.0, 12.0, _loguniform(rng, 0.5, 50.0))
    return Scene(eps.astype(np.float32), sig.astype(np.float32), seed,
                 name or f"disks{n_disks}_boxes{n_boxes}_lines{n_lines}_{S}")


def config2(seed: int = 2) -> Scene:
    """512x512: 32 disks, 64 opaque boxes (sigma 50), fog 0.05 * noise."""
    return scene_like_512(512, seed, 32, 64, name="disks32_boxes64_fog_512")


def config3(seed: int = 3) -> Scene:
    """1024x1024: 128 disks, 256 opaque boxes, 32 thin lines (sigma 100), fog."""
    return scene_like_512(1024, seed, 128, 256, n_lines=32,
                          name="disks128_boxes256_lines32_fog_1024")


def config4(seed: int = 4) -> Scene:
    """256x256 hidden target scene: 16 disks, 32 boxes of per-pixel sigma ~ U[0,5],
    fog 0.05 * noise."""
    return scene_like_512(256, seed, 16, 32, box_sigma="u05",
                          name="disks16_boxes32_fog_256")


def config5(seed: int = 5, count: int = 64, log2_sizes=(7, 8, 9, 10)) -> list:
    """``count`` scenes with log2 size uniform over ``log2_sizes``; scene i uses
    seed 5000+i and the 512x512 recipe at counts proportional to area."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(log2_sizes), size=count)
    out = []
    for i, n in enumerate(ns):
        S = 1 << int(n)
        scale = (S * S) / (512 * 512)
        nd = max(1, int(round(32 * scale)))
        nb = max(1, int(round(64 * scale)))
        out.append(scene_like_512(S, 5000 + i, nd, nb, name=f"batch{i}_{S}"))
    return out
