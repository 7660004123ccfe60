"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke run.

This module only *draws* inputs: uniform grids, analytic densities and seeded
Gaussian-mixture wave functions shaped like the workloads the paper studies
(Sec. 3.1, Examples 1 and 2; Sec. 3.2-3.3 initial data).  It contains none of
the potential solver's arithmetic, so both the FP64 oracle and the GPU path can
be fed from it without sharing any solver code.

Grid convention (Sec. 3, first paragraph): a square box [-L, L)^2 with N points
per side, spacing h = 2L/N, x_n = -L + n h for n = 0..N-1 (the periodic point
x = L is not stored).  Arrays are indexed [iy][ix] (x fastest), float64.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "grid_1d",
    "grid_2d",
    "gaussian_density",
    "paper_gaussian_density",
    "arkadiev_density",
    "MixtureSpec",
    "draw_mixture",
    "mixture_wave",
    "mixture_density",
    "batch_sides",
    "batch_members",
    "dsii_initial",
    "random_directions",
]


def grid_1d(n: int, half_width: float) -> tuple[np.ndarray, float]:
    """Points -L + n h, n = 0..N-1, and the spacing h = 2L/N."""
    h = 2.0 * half_width / n
    return -half_width + h * np.arange(n, dtype=np.float64), h


def grid_2d(n: int, half_width: float) -> tuple[np.ndarray, np.ndarray, float]:
    """Meshgrid (X, Y) indexed [iy][ix] plus the spacing."""
    x, h = grid_1d(n, half_width)
    y_mesh, x_mesh = np.meshgrid(x, x, indexing="ij")
    return x_mesh, y_mesh, h


def gaussian_density(n: int, half_width: float, amplitude: float = 1.0,
                     a: float = 1.0) -> np.ndarray:
    """rho = amplitude * exp(-a (x^2 + y^2)); a = 1 is the small FP64 case
    (64 x 64 over [-8, 8)^2)."""
    x_mesh, y_mesh, _ = grid_2d(n, half_width)
    return amplitude * np.exp(-a * (x_mesh ** 2 + y_mesh ** 2))


def paper_gaussian_density(n: int, half_width: float) -> np.ndarray:
    """Example 1 of Sec. 3.1: rho = pi exp(-pi^2 (x^2 + y^2))."""
    return gaussian_density(n, half_width, amplitude=math.pi, a=math.pi ** 2)


def arkadiev_density(n: int, half_width: float) -> np.ndarray:
    """Example 2 of Sec. 3.1: rho = 4 / ((x+1)^2 + y^2 + 1)^2."""
    x_mesh, y_mesh, _ = grid_2d(n, half_width)
    s = (x_mesh + 1.0) ** 2 + y_mesh ** 2 + 1.0
    return 4.0 / s ** 2


@dataclasses.dataclass(frozen=True)
class MixtureSpec:
    """u(x, y) = sum_i exp(-((x-cx_i)/wx_i)^2 - ((y-cy_i)/wy_i)^2 + i phase_i)."""
    cx: np.ndarray
    cy: np.ndarray
    wx: np.ndarray
    wy: np.ndarray
    phase: np.ndarray

    @property
    def count(self) -> int:
        return int(self.cx.shape[0])


def draw_mixture(seed: int, count: int = 8, centre_range: float = 6.0,
                 width_range: tuple[float, float] = (0.5, 2.0)) -> MixtureSpec:
    """Seeded anisotropic complex Gaussian mixture.

    Draw order (numpy default_rng(seed)): centres cx, cy ~ U[-r, r]; then widths
    wx, wy ~ U[w0, w1]; then phases ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    cx = rng.uniform(-centre_range, centre_range, count)
    cy = rng.uniform(-centre_range, centre_range, count)
    wx = rng.uniform(width_range[0], width_range[1], count)
    wy = rng.uniform(width_range[0], width_range[1], count)
    phase = rng.uniform(0.0, 2.0 * math.pi, count)
    return MixtureSpec(cx, cy, wx, wy, phase)


def mixture_wave(n: int, half_width: float, spec: MixtureSpec) -> np.ndarray:
    """Complex wave function u on the grid (complex128)."""
    x, _ = grid_1d(n, half_width)
    u = np.zeros((n, n), dtype=np.complex128)
    for i in range(spec.count):
        gx = np.exp(-((x - spec.cx[i]) / spec.wx[i]) ** 2)
        gy = np.exp(-((x - spec.cy[i]) / spec.wy[i]) ** 2)
        u += np.exp(1j * spec.phase[i]) * np.outer(gy, gx)
    return u


def mixture_density(n: int, half_width: float, spec: MixtureSpec) -> np.ndarray:
    """rho = |u|^2 built in float64."""
    u = mixture_wave(n, half_width, spec)
    return (u.real ** 2 + u.imag ** 2).astype(np.float64)


BATCH_SIDES = (128, 256, 512, 1024)


def batch_sides(seed: int = 1, count: int = 256) -> np.ndarray:
    """Grid sides of the uneven batch, uniform over {128, 256, 512, 1024}."""
    rng = np.random.default_rng(seed)
    return np.asarray(BATCH_SIDES, dtype=np.int64)[rng.integers(0, 4, count)]


def batch_members(seed: int = 1, count: int = 256, spacing: float = 1.0 / 32.0):
    """Members of the uneven batch: (side, half_width, MixtureSpec) per member.

    Each box is scaled so that the spacing is fixed (h = 1/32, so L = N/64); the
    8-Gaussian mixture law of the single 2048^2 case is scaled self-similarly
    (centres in [-0.375 L, 0.375 L]^2, widths in [0.5, 2] * L/16)."""
    sides = batch_sides(seed, count)
    rng = np.random.default_rng(seed + 1000)
    out = []
    for n in sides:
        half = 0.5 * float(n) * spacing
        member_seed = int(rng.integers(0, 2 ** 31 - 1))
        base = draw_mixture(member_seed, 8, 0.375 * half, (0.5, 2.0))
        scale = half / 16.0
        spec = MixtureSpec(base.cx, base.cy, base.wx * scale, base.wy * scale,
                           base.phase)
        out.append((int(n), half, spec))
    return out


def dsii_initial(n: int, half_width: float) -> np.ndarray:
    """u0 = exp(-(x^2 + 2 y^2)) (complex128), the time-stepping initial datum."""
    x_mesh, y_mesh, _ = grid_2d(n, half_width)
    return np.exp(-(x_mesh ** 2 + 2.0 * y_mesh ** 2)).astype(np.complex128)


def random_directions(n: int, seeds, like: np.ndarray | None = None):
    """Standard-normal directions (one per seed), optionally rescaled to the
    Frobenius norm of `like`."""
    out = []
    for s in seeds:
        v = np.random.default_rng(int(s)).standard_normal((n, n))
        if like is not None:
            v *= np.linalg.norm(like) / np.linalg.norm(v)
        out.append(v)
    return out
