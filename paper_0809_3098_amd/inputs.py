"""Seeded synthetic inputs shared by the GPU path's callers and the tests.

This module holds no arithmetic of the method: it only draws or tabulates
initial fields, which both the HIP path and the oracle then receive as plain
float64 arrays indexed [j, i] (x fastest, lid on the last row).
"""
from __future__ import annotations

import numpy as np


def zeros(n: int) -> np.ndarray:
    """Fluid at rest: omega = 0 everywhere, walls included."""
    return np.zeros((n, n), dtype=np.float64)


def noise_omega0(n: int, amplitude: float = 1e-3, seed: int = 0) -> np.ndarray:
    """Gaussian-noise initial vorticity on interior nodes, zero on the walls.

    ``amplitude * default_rng(seed).standard_normal((n-2, n-2))`` in [j, i]
    order, used to probe steadiness of the high-Re flow.
    """
    w = np.zeros((n, n), dtype=np.float64)
    w[1:-1, 1:-1] = amplitude * np.random.default_rng(seed).standard_normal((n - 2, n - 2))
    return w


def random_field(n: int, seed: int, scale: float = 1.0, zero_walls: bool = False) -> np.ndarray:
    """Uniform(-scale, scale) field for operator-level parity tests."""
    f = scale * (2.0 * np.random.default_rng(seed).random((n, n)) - 1.0)
    if zero_walls:
        f[0, :] = f[-1, :] = f[:, 0] = f[:, -1] = 0.0
    return f


def smooth_omega0(n: int, amplitude: float = 0.1) -> np.ndarray:
    """Vorticity of psi = amplitude sin^2(pi x) sin^2(pi y), tabulated on nodes.

    That psi vanishes with its normal derivative on every wall, so this is a
    smooth start compatible with no-slip walls.
    """
    x = np.arange(n, dtype=np.float64) / (n - 1)
    X, Y = np.meshgrid(x, x, indexing="xy")
    sx, sy = np.sin(np.pi * X), np.sin(np.pi * Y)
    return -2.0 * amplitude * np.pi**2 * (np.cos(2 * np.pi * X) * sy**2
                                          + np.cos(2 * np.pi * Y) * sx**2)
