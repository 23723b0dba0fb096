"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds no arithmetic of the method: it only draws positions,
species, cells and weight tensors from fixed seeds and describes the order
in which the weight tensors are packed into one flat float32 blob.  Both the
oracle (``oracle/``) and the GPU library parse that blob with their own code.

Workloads (synthetic stand-ins for the paper's dense condensed-phase cells;
the paper's Li3PO4 / SiOx / Pt-TiO2 structures are not available):

* ``small``    128 atoms, cubic 11.5 A box, 2 species, l_max=1, C=32, T=K=2.
* ``mpdp``     13,824 atoms (24^3 lattice), 3 species, l_max=2, C=64, T=6;
               evaluated at K=6 and K=2 (message-passing depth pruning,
               Methods "Message Passing Depth Pruning").
* ``bulk1m``   1,000,000 atoms (100^3 lattice), l_max=2, C=128, T=K=2.
* ``slab8m``   one eighth-slab share of an 8,000,000-atom box (200^3
               lattice) with a halo of depth K*r_cut (Methods "Graph
               Partitioning", stage 1 grid split along x); a 20,000-atom
               downscale (200 x 10 x 10 lattice) for the partition rule check.
* ``batch512`` 512 independent small periodic cells of 8..512 atoms.

Density 0.085 atoms/A^3 gives a simple-cubic lattice constant
a = 0.085**(-1/3) = 2.27437 A; every lattice workload adds N(0, 0.1 A)
jitter per coordinate.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Tuple

import numpy as np

DENSITY = 0.085                      # atoms / A^3
LATTICE_A = DENSITY ** (-1.0 / 3.0)  # 2.27437 A
JITTER = 0.1                         # A, std of the per-coordinate jitter


@dataclasses.dataclass(frozen=True)
class HParams:
    """Hyper-parameters of the equivariant message-passing potential."""
    n_species: int
    n_layers: int          # T: layers present in the weight blob
    l_max: int
    channels: int
    n_basis: int = 8
    envelope_p: int = 6
    radial_hidden: int = 64
    r_cut: float = 5.0
    avg_neighbors: float = 44.0

    @property
    def inv_avg_neighbors(self) -> float:
        return 1.0 / self.avg_neighbors


@dataclasses.dataclass
class System:
    """One periodic (or partly periodic) structure.

    ``cell`` rows are lattice vectors (A).  ``n_owned`` atoms come first;
    the energy is summed over them only (root atoms of a partition).
    """
    positions: np.ndarray   # [N,3] float64
    species: np.ndarray     # [N] int32
    cell: np.ndarray        # [3,3] float64
    pbc: np.ndarray         # [3] bool
    n_owned: int

    @property
    def n_atoms(self) -> int:
        return int(self.positions.shape[0])


# --------------------------------------------------------------------------
# weight blob layout
# --------------------------------------------------------------------------

def _count_paths(l_in: List[int], l_max: int) -> int:
    """Number of (l1,l2,l3) triples with l1 in l_in, l2,l3 <= l_max, l1+l2+l3
    even and |l1-l2| <= l3 <= l1+l2.  Only the count is needed here, to size
    the radial-MLP output tensor of each layer."""
    n = 0
    for l1 in l_in:
        for l2 in range(l_max + 1):
            for l3 in range(l_max + 1):
                if (l1 + l2 + l3) % 2 == 0 and abs(l1 - l2) <= l3 <= l1 + l2:
                    n += 1
    return n


def weight_layout(hp: HParams) -> List[Tuple[str, Tuple[int, ...], int]]:
    """(name, shape, fan_in) of every tensor, in blob order.

    Order: W_emb; then for each layer t = 1..T: W_up for every input degree
    l (only l=0 at t=1), W1, W2, W3, W_down for l = 0..l_max; then w_read and
    e0.  Every matrix maps rows (inputs) to columns (outputs).  W_down for
    l=0 has C*(1+l_max) columns: C scalar features followed by one gate block
    of C per degree l >= 1.  W3 has P_t*C columns, path-major.
    """
    C, H, nb, L = hp.channels, hp.radial_hidden, hp.n_basis, hp.l_max
    out = [("W_emb", (hp.n_species, C), 1)]
    for t in range(1, hp.n_layers + 1):
        l_in = [0] if t == 1 else list(range(L + 1))
        for l in l_in:
            out.append((f"L{t}.W_up{l}", (C, C), C))
        out.append((f"L{t}.W1", (nb, H), nb))
        out.append((f"L{t}.W2", (H, H), H))
        out.append((f"L{t}.W3", (H, _count_paths(l_in, L) * C), H))
        out.append((f"L{t}.W_down0", (C, C * (1 + L)), C))
        for l in range(1, L + 1):
            out.append((f"L{t}.W_down{l}", (C, C), C))
    out.append(("w_read", (C,), C))
    out.append(("e0", (hp.n_species,), 0))
    return out


def weights_count(hp: HParams) -> int:
    return sum(int(np.prod(s)) for _, s, _ in weight_layout(hp))


def make_weights(hp: HParams, seed: int, e0: np.ndarray | None = None) -> np.ndarray:
    """Flat float32 blob: each tensor ~ N(0, 1/fan_in) drawn in float64 from
    numpy's PCG64 in blob order, then stored as float32.  ``e0`` (per-species
    energy offsets) is zero unless given."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape, fan_in in weight_layout(hp):
        if name == "e0":
            v = np.zeros(shape) if e0 is None else np.asarray(e0, dtype=np.float64)
        else:
            v = rng.standard_normal(shape) / math.sqrt(fan_in)
        parts.append(np.asarray(v, dtype=np.float64).astype(np.float32).ravel())
    return np.concatenate(parts)


# --------------------------------------------------------------------------
# positions / species
# --------------------------------------------------------------------------

def lattice_positions(nx: int, ny: int, nz: int, a: float, seed: int,
                      jitter: float = JITTER) -> np.ndarray:
    """Simple-cubic lattice (x fastest) plus N(0, jitter) per coordinate."""
    rng = np.random.default_rng(seed)
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    grid = np.stack([ix.ravel(order="F"), iy.ravel(order="F"), iz.ravel(order="F")], axis=1)
    pos = (grid.astype(np.float64) + 0.5) * a
    pos += rng.standard_normal(pos.shape) * jitter
    return pos


def species_by_fraction(n: int, fractions, seed: int) -> np.ndarray:
    """Exact counts round(n*f) (the last species takes the remainder),
    assigned by a seeded permutation."""
    counts = [int(round(n * f)) for f in fractions[:-1]]
    counts.append(n - sum(counts))
    lab = np.concatenate([np.full(c, s, dtype=np.int32) for s, c in enumerate(counts)])
    rng = np.random.default_rng(seed)
    return lab[rng.permutation(n)].astype(np.int32)


def cubic_cell(L: float) -> np.ndarray:
    return np.diag([L, L, L]).astype(np.float64)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

HP_SMALL = HParams(n_species=2, n_layers=2, l_max=1, channels=32)
HP_MPDP = HParams(n_species=3, n_layers=6, l_max=2, channels=64)
HP_BULK = HParams(n_species=3, n_layers=2, l_max=2, channels=128)
HP_BATCH = HParams(n_species=3, n_layers=2, l_max=2, channels=64)
SPECIES_FRACTIONS = (0.5, 0.3, 0.2)


def small_system(seed_pos: int = 101, seed_species: int = 102) -> System:
    """128 of the 216 sites of a 6x6x6 simple-cubic grid in an 11.5 A box,
    chosen by a seeded permutation, plus jitter; species i.i.d. U{0,1}."""
    L = 11.5
    sites = lattice_positions(6, 6, 6, L / 6.0, seed_pos, jitter=0.0)
    rng = np.random.default_rng(seed_pos)
    keep = np.sort(rng.permutation(216)[:128])
    pos = sites[keep] + rng.standard_normal((128, 3)) * JITTER
    sp = np.random.default_rng(seed_species).integers(0, 2, size=128).astype(np.int32)
    return System(pos, sp, cubic_cell(L), np.array([True, True, True]), 128)


def bulk_system(n_side: int, seed_pos: int, seed_species: int) -> System:
    """n_side^3 jittered simple-cubic lattice at density 0.085, 3 species
    with fractions 0.5/0.3/0.2 (exact counts)."""
    n = n_side ** 3
    pos = lattice_positions(n_side, n_side, n_side, LATTICE_A, seed_pos)
    sp = species_by_fraction(n, SPECIES_FRACTIONS, seed_species)
    return System(pos, sp, cubic_cell(n_side * LATTICE_A), np.array([True, True, True]), n)


def mpdp_system() -> System:
    return bulk_system(24, 201, 202)


def bulk1m_system() -> System:
    return bulk_system(100, 301, 302)


def slab_full_system(nx: int, ny: int, nz: int, seed_pos: int, seed_species: int) -> System:
    """Full periodic box for the partition workloads (x is the split axis)."""
    n = nx * ny * nz
    pos = lattice_positions(nx, ny, nz, LATTICE_A, seed_pos)
    sp = species_by_fraction(n, SPECIES_FRACTIONS, seed_species)
    cell = np.diag([nx * LATTICE_A, ny * LATTICE_A, nz * LATTICE_A]).astype(np.float64)
    return System(pos, sp, cell, np.array([True, True, True]), n)


def slab_downscale_full() -> System:
    """20,000-atom downscale of the 8M-atom partitioned box."""
    return slab_full_system(200, 10, 10, 401, 402)


WEIGHT_SEEDS: Dict[str, int] = {"small": 103, "mpdp": 203, "bulk1m": 303,
                                "slab8m": 403, "batch512": 503}


def batch_structures(n_struct: int = 512, seed: int = 501, seed_species: int = 502,
                     n_min: int = 8, n_max: int = 512, d_min: float = 1.5) -> List[System]:
    """Independent periodic cells of uneven size at density 0.085.

    N ~ U{n_min..n_max}; volume V = N/0.085.  If V >= 216 A^3 the three
    orthorhombic sides are drawn in [6, 20] A by rejection so that their
    product is V; otherwise the cell is a cube of side V^(1/3).  Positions by
    seeded random sequential addition with minimum distance d_min (minimum
    image); species i.i.d. categorical(0.5, 0.3, 0.2)."""
    rng = np.random.default_rng(seed)
    rng_sp = np.random.default_rng(seed_species)
    out = []
    for _ in range(n_struct):
        n = int(rng.integers(n_min, n_max + 1))
        V = n / DENSITY
        if V >= 216.0:
            while True:
                a = rng.uniform(6.0, 20.0)
                b = rng.uniform(6.0, 20.0)
                c = V / (a * b)
                if 6.0 <= c <= 20.0:
                    break
            sides = np.array([a, b, c])
        else:
            sides = np.full(3, V ** (1.0 / 3.0))
        pos = np.zeros((n, 3))
        k = 0
        tries = 0
        while k < n:
            p = rng.uniform(0.0, 1.0, 3) * sides
            if k:
                dd = pos[:k] - p
                dd -= np.round(dd / sides) * sides
                if np.min(np.einsum("ij,ij->i", dd, dd)) < d_min * d_min:
                    tries += 1
                    if tries > 200000:
                        raise RuntimeError("random sequential addition did not converge")
                    continue
            pos[k] = p
            k += 1
        sp = rng_sp.choice(3, size=n, p=list(SPECIES_FRACTIONS)).astype(np.int32)
        out.append(System(pos, sp, np.diag(sides).astype(np.float64),
                          np.array([True, True, True]), n))
    return out


# masses (amu) of a three-species Li3PO4 stand-in (Li, P, O), for MD runs
MASSES_LPO = (6.94, 30.973762, 15.999)


def velocities(n: int, sigma: float, seed: int) -> np.ndarray:
    """Initial velocities for MD tests: N(0, sigma) per component (A/fs)."""
    return np.random.default_rng(seed).standard_normal((n, 3)) * sigma


def rejitter(pos: np.ndarray, seed: int, amp: float = 0.01) -> np.ndarray:
    """Small seeded displacement (+-amp, uniform) applied between timed calls
    so that no neighbour-list cache can help."""
    rng = np.random.default_rng(seed)
    return pos + rng.uniform(-amp, amp, pos.shape)
