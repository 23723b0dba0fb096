"""Coupling tensors and path lists (oracle).

For degrees (l1, l2, l3) the real Gaunt tensor is
    G[m1, m2, m3] = integral over the unit sphere of Y^l1_m1 Y^l2_m2 Y^l3_m3
with the component-normalised real harmonics of ``oracle.sh``.  The
coupling tensor is its Frobenius normalisation C = G / ||G||_F.  Only
"natural parity" triples are used: l1 + l2 + l3 even and
|l1 - l2| <= l3 <= l1 + l2, so that the energy is invariant under all of
O(3).

The integral is taken by product quadrature: Gauss-Legendre in cos(theta)
(8 nodes, exact for polynomials of degree <= 15) times the uniform rule in
phi (16 nodes, exact for trigonometric degree <= 15); the integrand has
degree <= 6, so the quadrature is exact up to rounding.
"""
from __future__ import annotations

from functools import lru_cache
from typing import List, Tuple

import numpy as np

from .sh import real_sh


@lru_cache(maxsize=None)
def _quadrature():
    zs, wz = np.polynomial.legendre.leggauss(8)
    nphi = 16
    phis = 2.0 * np.pi * np.arange(nphi) / nphi
    Z, PHI = np.meshgrid(zs, phis, indexing="ij")
    W = np.repeat(wz[:, None], nphi, axis=1) * (2.0 * np.pi / nphi)
    st = np.sqrt(1.0 - Z * Z)
    u = np.stack([st * np.cos(PHI), st * np.sin(PHI), Z], axis=-1).reshape(-1, 3)
    return u, W.reshape(-1)


def gaunt_tensor(l1: int, l2: int, l3: int) -> np.ndarray:
    u, w = _quadrature()
    Y = real_sh(u, 2)
    b1, b2, b3 = (slice(l * l, (l + 1) * (l + 1)) for l in (l1, l2, l3))
    return np.einsum("q,qa,qb,qc->abc", w, Y[:, b1], Y[:, b2], Y[:, b3])


@lru_cache(maxsize=None)
def coupling_tensor(l1: int, l2: int, l3: int) -> np.ndarray:
    G = gaunt_tensor(l1, l2, l3)
    C = G / np.linalg.norm(G)
    C.setflags(write=False)
    return C


def natural(l1: int, l2: int, l3: int) -> bool:
    return (l1 + l2 + l3) % 2 == 0 and abs(l1 - l2) <= l3 <= l1 + l2


def layer_paths(t: int, l_max: int) -> List[Tuple[int, int, int]]:
    """All paths of layer t (1-based) in weight order: l1 over the input
    degrees ({0} at t = 1, else 0..l_max), then l2, then l3, ascending."""
    l_in = [0] if t == 1 else list(range(l_max + 1))
    return [(l1, l2, l3) for l1 in l_in for l2 in range(l_max + 1)
            for l3 in range(l_max + 1) if natural(l1, l2, l3)]


def live_paths(t: int, K: int, l_max: int) -> List[Tuple[int, int]]:
    """(index into layer_paths, path) of the paths that influence the
    energy when K layers are evaluated: all of them below the last layer;
    at layer K only those ending in l3 = 0 (only scalars are read out)."""
    out = []
    for idx, p in enumerate(layer_paths(t, l_max)):
        if t < K or p[2] == 0:
            out.append((idx, p))
    return out
