"""Molecular dynamics around the oracle's energy and forces (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The step is the BAOAB splitting of Langevin dynamics (Leimkuhler and
Matthews, "Rational construction of stochastic numerical methods for
molecular sampling", 2013); the paper's MD runs use Langevin dynamics
(results, Li3PO4 throughput and quench).  One step of length dt:
  B: v <- v + (dt/2) F/m
  A: x <- x + (dt/2) v
  O: v <- c1 v + sqrt(1 - c1^2) sqrt(kB T / m) xi,   c1 = exp(-gamma dt)
  A: x <- x + (dt/2) v
     F <- F(x)
  B: v <- v + (dt/2) F/m
With gamma = 0 the O step is the identity and the step is velocity Verlet.
Units: Angstrom, fs, eV, amu, K; F/m in eV/(Angstrom amu) times the factor
e / amu (in SI) * 1e-20 gives Angstrom / fs^2.

xi: three standard normal numbers per atom and step, from Philox4x32-10
(Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11) with the 64-bit seed as the key and the counter (atom index as two
32-bit words, step index as two words), and the Box-Muller transform of
u0 = (w0 + 1)/2^32, u1 = (w1 + 0.5)/2^32 (first pair) and w2, w3 likewise.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .model import evaluate

ELEMENTARY_CHARGE = 1.602176634e-19   # C (exact in SI)
ATOMIC_MASS_UNIT = 1.66053906660e-27  # kg
BOLTZMANN_EV = 8.617333262e-5         # eV / K
# (eV / Angstrom) / amu -> Angstrom / fs^2: (J / 1e-10 m) / kg = m/s^2 = 1e-20 Angstrom / fs^2
ACCEL = ELEMENTARY_CHARGE / (1e-10 * ATOMIC_MASS_UNIT) * 1e-20

_M0, _M1 = 0xD2511F53, 0xCD9E8D57      # Philox4x32 multipliers
_W0, _W1 = 0x9E3779B9, 0xBB67AE85      # Weyl key increments
_MASK = 0xFFFFFFFF


def philox4x32_10(counter, key):
    """Ten Philox4x32 rounds on the counter (4 uint32) with the key (2 uint32);
    each round multiplies words 0 and 2 by the two constants (64-bit product),
    and the new words are (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
    lo(M0 c0)); the key advances by the Weyl constants between rounds."""
    c0, c1, c2, c3 = (int(x) & _MASK for x in counter)
    k0, k1 = (int(x) & _MASK for x in key)
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & _MASK, p1 & _MASK, ((p0 >> 32) ^ c3 ^ k1) & _MASK, p0 & _MASK
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return c0, c1, c2, c3


def normals3(seed: int, atom: int, step: int) -> np.ndarray:
    """Three N(0,1) numbers of (atom, step): Box-Muller on the four words."""
    key = (seed & _MASK, (seed >> 32) & _MASK)
    w = philox4x32_10((atom & _MASK, (atom >> 32) & _MASK, step & _MASK, (step >> 32) & _MASK), key)
    two32 = 4294967296.0
    u0, u1 = (w[0] + 1.0) / two32, (w[1] + 0.5) / two32
    u2, u3 = (w[2] + 1.0) / two32, (w[3] + 0.5) / two32
    r0, r1 = math.sqrt(-2.0 * math.log(u0)), math.sqrt(-2.0 * math.log(u2))
    return np.array([r0 * math.cos(2.0 * math.pi * u1), r0 * math.sin(2.0 * math.pi * u1),
                     r1 * math.cos(2.0 * math.pi * u3)])


@dataclasses.dataclass
class Trajectory:
    positions: np.ndarray    # [n_steps+1, N, 3] (entry 0: start)
    velocities: np.ndarray   # [n_steps+1, N, 3]
    forces: np.ndarray       # [n_steps+1, N, 3]
    epot: np.ndarray         # [n_steps] root-atom potential energy after each step (eV)
    ekin: np.ndarray         # [n_steps] kinetic energy after each step (eV)


def kinetic_energy(velocities, masses_per_atom) -> float:
    """sum_i m_i |v_i|^2 / 2 in eV (velocities in Angstrom / fs)."""
    v = np.asarray(velocities, dtype=np.float64)
    return float(0.5 * np.sum(masses_per_atom[:, None] * v * v) / ACCEL)


def run(positions, velocities, species, masses, cell, pbc, blob, hp, K, dt: float, n_steps: int,
        friction: float = 0.0, temperature: float = 0.0, seed: int = 0, force_fn=None) -> Trajectory:
    """n_steps BAOAB steps (velocity Verlet for friction 0) from (positions,
    velocities) with the oracle's forces (or ``force_fn(x) -> (E, F)``)."""
    x = np.array(positions, dtype=np.float64)
    v = np.array(velocities, dtype=np.float64)
    sp = np.asarray(species)
    m = np.asarray(masses, dtype=np.float64)[sp]
    N = x.shape[0]

    def forces_at(xx):
        if force_fn is not None:
            return force_fn(xx)
        r = evaluate(xx, sp, cell, pbc, blob, hp, K=K)
        return r.energy, r.forces

    _, F = forces_at(x)
    c1 = math.exp(-friction * dt)
    c2 = math.sqrt(1.0 - c1 * c1)
    kT = BOLTZMANN_EV * temperature
    xs, vs, fs, ep, ek = [x.copy()], [v.copy()], [F.copy()], [], []
    for step in range(n_steps):
        a = ACCEL * F / m[:, None]
        v = v + 0.5 * dt * a                                   # B
        x = x + 0.5 * dt * v                                   # A
        if friction != 0.0:                                    # O
            sig = np.sqrt(kT * ACCEL / m)
            xi = np.stack([normals3(seed, i, step) for i in range(N)])
            v = c1 * v + c2 * sig[:, None] * xi
        x = x + 0.5 * dt * v                                   # A
        E, F = forces_at(x)
        v = v + 0.5 * dt * ACCEL * F / m[:, None]              # B
        xs.append(x.copy())
        vs.append(v.copy())
        fs.append(F.copy())
        ep.append(E)
        ek.append(kinetic_energy(v, m))
    return Trajectory(np.array(xs), np.array(vs), np.array(fs), np.array(ep), np.array(ek))
