"""Brute-force O(N^2) periodic neighbour list (oracle).

An edge is an ordered triple (i, j, S), S in Z^3, with
    r = x_j - x_i + S . cell          (cell rows are lattice vectors)
and |r| < r_cut strictly; (i, i, 0) is excluded.  i receives, j sends.

The membership test is evaluated in float64 with one rounding per operation
and a fixed order, so that any other implementation that uses the same
order decides every pair identically:
    s_k  = (S_0*cell[0,k] + S_1*cell[1,k]) + S_2*cell[2,k]
    dx_k = (x_j[k] - x_i[k]) + s_k
    d2   = (dx_0*dx_0 + dx_1*dx_1) + dx_2*dx_2
    edge iff d2 < r_cut*r_cut
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def perpendicular_widths(cell: np.ndarray) -> np.ndarray:
    """Distance between opposite faces of the cell, per lattice direction."""
    cell = np.asarray(cell, dtype=np.float64)
    vol = abs(np.linalg.det(cell))
    w = np.empty(3)
    for k in range(3):
        a, b = cell[(k + 1) % 3], cell[(k + 2) % 3]
        w[k] = vol / np.linalg.norm(np.cross(a, b))
    return w


def _pair_test(pos, cell, r_cut, ii, jj, S):
    """The exact float64 predicate above on index arrays ii, jj and integer
    shifts S [n,3]; returns the boolean mask."""
    Sf = S.astype(np.float64)
    s = (Sf[:, 0:1] * cell[0][None, :] + Sf[:, 1:2] * cell[1][None, :]) + Sf[:, 2:3] * cell[2][None, :]
    dx = (pos[jj] - pos[ii]) + s
    d2 = (dx[:, 0] * dx[:, 0] + dx[:, 1] * dx[:, 1]) + dx[:, 2] * dx[:, 2]
    keep = d2 < r_cut * r_cut
    keep &= ~((ii == jj) & np.all(S == 0, axis=1))
    return keep


def neighbor_list(positions, cell, pbc, r_cut: float, chunk: int = 256):
    """All edges (i, j, S), sorted by (i, j, S_x, S_y, S_z).

    If the cell is orthorhombic and every periodic direction is at least
    2*r_cut wide, at most one image of each pair can lie within r_cut, and it
    is the minimum image: S_k = -round((x_j - x_i)_k / L_k).  Otherwise every
    image with |S_k| <= ceil(r_cut / width_k) is tested (self images included).
    Returns (i int64[E], j int64[E], S int64[E,3]).
    """
    pos = np.asarray(positions, dtype=np.float64)
    cell = np.asarray(cell, dtype=np.float64)
    pbc = np.asarray(pbc, dtype=bool)
    n = pos.shape[0]
    widths = perpendicular_widths(cell) if np.any(pbc) else np.full(3, np.inf)
    ortho = np.count_nonzero(cell - np.diag(np.diag(cell))) == 0
    minimum_image = ortho and all((not pbc[k]) or widths[k] >= 2.0 * r_cut for k in range(3))
    I, J, SS = [], [], []
    if minimum_image:
        L = np.diag(cell)
        jj_all = np.arange(n)
        for i0 in range(0, n, chunk):
            i1 = min(n, i0 + chunk)
            dx = pos[None, :, :] - pos[i0:i1, None, :]            # x_j - x_i
            S = np.zeros(dx.shape, dtype=np.int64)
            for k in range(3):
                if pbc[k]:
                    S[:, :, k] = -np.round(dx[:, :, k] / L[k]).astype(np.int64)
            Sf = S.astype(np.float64)
            s = ((Sf[..., 0:1] * cell[0] + Sf[..., 1:2] * cell[1]) + Sf[..., 2:3] * cell[2])
            r = dx + s
            d2 = (r[..., 0] * r[..., 0] + r[..., 1] * r[..., 1]) + r[..., 2] * r[..., 2]
            keep = d2 < r_cut * r_cut
            ii = np.arange(i0, i1)
            keep[ii - i0, ii] &= ~np.all(S[ii - i0, ii] == 0, axis=1)
            a, b = np.nonzero(keep)
            I.append(a + i0); J.append(jj_all[b]); SS.append(S[a, b])
    else:
        nimg = [int(math.ceil(r_cut / widths[k])) if pbc[k] else 0 for k in range(3)]
        images = np.array(list(itertools.product(*[range(-m, m + 1) for m in nimg])), dtype=np.int64)
        for i0 in range(0, n, chunk):
            i1 = min(n, i0 + chunk)
            for S0 in images:
                ii = np.repeat(np.arange(i0, i1), n)
                jj = np.tile(np.arange(n), i1 - i0)
                S = np.broadcast_to(S0, (ii.size, 3))
                keep = _pair_test(pos, cell, r_cut, ii, jj, S)
                I.append(ii[keep]); J.append(jj[keep]); SS.append(np.array(S[keep]))
    I = np.concatenate(I) if I else np.zeros(0, np.int64)
    J = np.concatenate(J) if J else np.zeros(0, np.int64)
    SS = np.concatenate(SS) if SS else np.zeros((0, 3), np.int64)
    order = np.lexsort((SS[:, 2], SS[:, 1], SS[:, 0], J, I))
    return I[order], J[order], SS[order]


def edge_vectors(positions, cell, i, j, S) -> np.ndarray:
    """r_e = (x_j - x_i) + S . cell in float64, same operation order as the
    membership test."""
    pos = np.asarray(positions, dtype=np.float64)
    cell = np.asarray(cell, dtype=np.float64)
    Sf = np.asarray(S, dtype=np.float64)
    s = (Sf[:, 0:1] * cell[0][None, :] + Sf[:, 1:2] * cell[1][None, :]) + Sf[:, 2:3] * cell[2][None, :]
    return (pos[j] - pos[i]) + s
