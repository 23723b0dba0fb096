"""Real spherical harmonics, component normalised (oracle).

For a unit vector u = (x, y, z), degrees l <= 2, m ordered -l..l:
    Y^0 = 1
    Y^1 = sqrt(3) * (y, z, x)
    Y^2 = (sqrt(15) x y, sqrt(15) y z, sqrt(5)/2 (3 z^2 - 1),
           sqrt(15) x z, sqrt(15)/2 (x^2 - y^2))
so that sum_m (Y^l_m)^2 = 2l+1 on the sphere.  Components are stored
flat, index l^2 + (m + l).
"""
from __future__ import annotations

import numpy as np

S3 = np.sqrt(3.0)
S5 = np.sqrt(5.0)
S15 = np.sqrt(15.0)


def real_sh(u: np.ndarray, l_max: int = 2) -> np.ndarray:
    u = np.asarray(u, dtype=np.float64)
    x, y, z = u[:, 0], u[:, 1], u[:, 2]
    cols = [np.ones_like(x)]
    if l_max >= 1:
        cols += [S3 * y, S3 * z, S3 * x]
    if l_max >= 2:
        cols += [S15 * x * y, S15 * y * z, 0.5 * S5 * (3.0 * z * z - 1.0),
                 S15 * x * z, 0.5 * S15 * (x * x - y * y)]
    return np.stack(cols, axis=1)


def real_sh_grad(u: np.ndarray, l_max: int = 2) -> np.ndarray:
    """dP/du [E, (l_max+1)^2, 3] of the polynomials above, taken as
    polynomials in (x, y, z) off the sphere."""
    u = np.asarray(u, dtype=np.float64)
    x, y, z = u[:, 0], u[:, 1], u[:, 2]
    o, zero = np.ones_like(x), np.zeros_like(x)
    rows = [[zero, zero, zero]]
    if l_max >= 1:
        rows += [[zero, S3 * o, zero], [zero, zero, S3 * o], [S3 * o, zero, zero]]
    if l_max >= 2:
        rows += [[S15 * y, S15 * x, zero],
                 [zero, S15 * z, S15 * y],
                 [zero, zero, 3.0 * S5 * z],
                 [S15 * z, zero, S15 * x],
                 [S15 * x, -S15 * y, zero]]
    return np.stack([np.stack(r, axis=1) for r in rows], axis=1)
