"""Graph partitioning with halos and output integration (oracle).

Methods, "Graph Partitioning", stage 1 (spatial grid): the scaled position
of each atom along the split axis is binned into P equal bins; the atoms of
bin p are the root ("owned") atoms of partition p.  Stage 2 extends each
root set so that every root atom keeps the K-hop neighbourhood it has in the
full structure.  ``slab_share`` uses a geometric halo: every periodic image
of every atom whose coordinate along the split axis lies within ``halo`` of
the slab (and outside it) is added as a ghost at its unwrapped position.  A
halo of depth K*r_cut contains the K-hop set (each hop is shorter than
r_cut), so root energies are exact.  ``bfs_share`` keeps exactly the K-hop
set (the paper's breadth-first expansion).

Methods, "Global Output Integration": the energy is the sum of root-atom
energies over partitions; for gradient (conservative) models the force is
the sum over partitions of the gradients of each partition's root energy,
and the stress decomposes the same way.  ``evaluate_partitioned`` applies
these rules: ghost rows of each partition's force array (partial forces on
ghost copies) are added to the atoms they copy.
"""
from __future__ import annotations

import numpy as np

from .model import evaluate
from .neighbors import neighbor_list


def slab_share(positions, species, cell, n_parts: int, part: int, halo: float, axis: int = 0):
    """Local system of one slab partition.

    Returns (local_positions, local_species, pbc, n_owned, global_index) with
    the owned atoms first (in increasing global index), then the ghost
    images.  The split axis becomes non-periodic; the cell must be
    orthorhombic.
    """
    pos = np.asarray(positions, dtype=np.float64)
    cell = np.asarray(cell, dtype=np.float64)
    Lx = cell[axis, axis]
    x = pos[:, axis] - np.floor(pos[:, axis] / Lx) * Lx          # wrapped into [0, Lx)
    frac = x / Lx
    b = np.minimum(np.floor(frac * n_parts).astype(np.int64), n_parts - 1)
    lo, hi = part * Lx / n_parts, (part + 1) * Lx / n_parts
    owned = np.flatnonzero(b == part)
    loc_pos = [pos[owned].copy()]
    loc_pos[0][:, axis] = x[owned]
    gidx = [owned]
    n_img = int(np.ceil(halo / Lx)) + 1
    for s in range(-n_img, n_img + 1):
        xs = x + s * Lx
        in_halo = ((xs >= lo - halo) & (xs < lo)) | ((xs >= hi) & (xs < hi + halo))
        if s == 0:
            in_halo &= (b != part)
        sel = np.flatnonzero(in_halo)
        p = pos[sel].copy()
        p[:, axis] = xs[sel]
        loc_pos.append(p)
        gidx.append(sel)
    lp = np.concatenate(loc_pos)
    gi = np.concatenate(gidx)
    pbc = np.array([True, True, True])
    pbc[axis] = False
    return lp, np.asarray(species)[gi].astype(np.int32), pbc, owned.size, gi


def hop_distance(positions, cell, pbc, roots, r_cut: float, K: int):
    """Graph distance from the root set in the neighbour graph at r_cut
    (number of edges on a shortest path), capped at K + 1: level h + 1 is the
    set of neighbours of level h not reached before (breadth-first search,
    Methods "Graph Partitioning", stage 2)."""
    pos = np.asarray(positions, dtype=np.float64)
    i, j, _ = neighbor_list(pos, cell, pbc, r_cut)
    hop = np.full(pos.shape[0], K + 1, dtype=np.int64)
    hop[np.asarray(roots, dtype=np.int64)] = 0
    for h in range(K):
        nxt = j[hop[i] == h]
        hop[nxt] = np.minimum(hop[nxt], h + 1)
    return hop


def bfs_share(positions, species, cell, n_parts: int, part: int, K: int, r_cut: float, axis: int = 0,
              pbc=(True, True, True)):
    """Local system of one slab partition with a graph halo (Methods "Graph
    Partitioning": stage 1 grid, stage 2 expansion of each subgraph by K
    hops).  The roots are those of ``slab_share``; the halo is every atom
    within K hops of a root in the neighbour graph of the whole structure,
    placed at its image within K*r_cut of the slab (each hop is shorter
    than r_cut), which is unique when the slab plus 2*K*r_cut fits in the
    cell.  Same row order as ``slab_share`` with halo K*r_cut, whose rows of
    atoms farther than K hops are dropped.  Returns (local_positions,
    local_species, pbc, n_owned, global_index)."""
    cell = np.asarray(cell, dtype=np.float64)
    Lx = cell[axis, axis]
    if Lx / n_parts + 2.0 * K * r_cut > Lx:
        raise ValueError("slab plus halo wider than the cell")
    lp, ls, lpbc, n_own, gi = slab_share(positions, species, cell, n_parts, part, K * r_cut, axis)
    hop = hop_distance(positions, cell, pbc, gi[:n_own], r_cut, K)
    keep = np.ones(lp.shape[0], dtype=bool)
    keep[n_own:] = hop[gi[n_own:]] <= K
    return lp[keep], ls[keep], lpbc, n_own, gi[keep]


def evaluate_partitioned(positions, species, cell, blob, hp, K: int, n_parts: int,
                         halo: float, axis: int = 0):
    """Sequential evaluation of all partitions (the paper's one-GPU mode)
    and integration of the outputs.  Returns (E, F, W, per_part) where
    per_part holds each partition's result and index map."""
    N = np.asarray(positions).shape[0]
    E = 0.0
    F = np.zeros((N, 3))
    W = np.zeros((3, 3))
    parts = []
    for p in range(n_parts):
        lp, ls, pbc, n_own, gi = slab_share(positions, species, cell, n_parts, p, halo, axis)
        res = evaluate(lp, ls, cell, pbc, blob, hp, K=K, n_owned=n_own)
        E += res.energy
        np.add.at(F, gi, res.forces)
        W += res.virial
        parts.append((res, gi, n_own))
    return E, F, W, parts


def local_cluster(positions, species, cell, center: int, radius: float, inner: float):
    """Non-periodic cluster around one atom of a periodic orthorhombic cell.

    Atoms within ``radius`` (minimum image) of ``center`` are unwrapped
    relative to it; those within ``inner`` come first (they are the owned
    atoms).  Returns (positions, species, n_owned, global_index, local index
    of the center).  With inner = K*r_cut and radius = 2*K*r_cut the owned
    atoms' energies are exact and the force on the center atom equals the
    full-system force (the center feels only atoms within K*r_cut through
    their energies, and those energies see only atoms within 2*K*r_cut).
    """
    pos = np.asarray(positions, dtype=np.float64)
    L = np.diag(np.asarray(cell, dtype=np.float64))
    dx = pos - pos[center]
    dx -= np.round(dx / L) * L
    dist = np.sqrt(np.sum(dx * dx, axis=1))
    a = np.flatnonzero(dist < inner)
    b = np.flatnonzero((dist >= inner) & (dist < radius))
    gi = np.concatenate([a, b])
    lp = pos[center] + dx[gi]
    loc_center = int(np.flatnonzero(gi == center)[0])
    return lp, np.asarray(species)[gi].astype(np.int32), a.size, gi, loc_center
